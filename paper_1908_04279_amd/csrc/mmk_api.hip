// C-ABI of the micro-step library: argument checks, workspace layout, launch sequencing.
// Every step of the method runs in the HIP kernels of motor.hip, psi.hip and adjoint.hip;
// this file only validates, carves the caller's workspace and enqueues work on the stream.
#include "../../include/mmk.h"
#include "consts.h"
#include "kernels.h"
#include "tape.h"
#include "force.h"
#include "r0.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace mmk;

namespace {

thread_local std::string g_create_error;
constexpr int kMaxTheta = 512;
constexpr int kMaxS = 512;
constexpr int kProfIds = 10;
constexpr int kMaxBlock = 16;  // micro-steps per temporally blocked motor launch
constexpr int kProfMax = 65536;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t M[2], psi[2], psi_tmp, m0, m0s, m1, Dxy, fpart, fblk, fexy, fcs, u, G, stress, mom, tab, partials, sums;
    size_t q0, r0part, r0scale, r0pool, r0seg, r0start, psiT, Mmarg;  // anchor-resolved model (rc > 0)
    size_t q01, r0slot, r0cpos;  // one anchor per block: run total pairs, slot and cell tables
    TapeLayout tape;
    size_t total;
    int psi_blocks;
};

int64_t n_psi(const mmk_params &p) { return (int64_t)p.nx * p.ny * p.ntheta; }
int64_t n_m(const mmk_params &p) { return n_psi(p) * p.ns; }
R0Plan r0_plan_of(const mmk_params &p, bool cells_only = false) {
    return plan_r0(p.nx, p.ny, p.ntheta, p.ns, p.lx, p.ly, p.L, p.rc, cells_only);
}
size_t esize(const mmk_params &p);
// Slots of the one-pass depleted sub-cycling (one anchor per block), for the parameters that can
// use it: depletion and motor sub-cycling.
R0Slots r0_slots_of(const mmk_params &p, const R0Plan &rp) {
    if (!(p.rc > 0 && p.m_total > 0 && p.motor_cfl > 0)) return R0Slots{};
    if ((int64_t)p.nx * p.ny * p.ntheta >= ((int64_t)1 << 31)) return R0Slots{};  // 32-bit psi offsets
    return plan_r0_slots(rp, esize(p));
}
size_t esize(const mmk_params &p) { return p.precision == MMK_FP32 ? 4 : 8; }

// Returns an error message, or empty when the parameters are usable.
std::string check_params(const mmk_params *p) {
    if (!p) return "params is NULL";
    if (p->nx < 1 || p->ny < 1) return "nx and ny must be >= 1";
    if (p->ntheta < 1) return "ntheta must be >= 1";
    if (p->ns < 1) return "ns must be >= 1";
    if (p->precision != MMK_FP32 && p->precision != MMK_FP64) return "precision must be MMK_FP64 or MMK_FP32";
    if (p->limiter != MMK_SUPERBEE && p->limiter != MMK_UPWIND1) return "limiter must be MMK_SUPERBEE or MMK_UPWIND1";
    const double vals[] = {p->lx, p->ly, p->L, p->k_on, p->k_off, p->v0, p->F, p->sigma_f, p->m_total,
                           p->motor_cfl, p->rc};
    for (double v : vals)
        if (!std::isfinite(v)) return "non-finite model parameter";
    if (p->lx <= 0 || p->ly <= 0 || p->L <= 0) return "lx, ly and L must be > 0";
    if (p->v0 < 0) return "v0 must be >= 0 (motors walk towards s = L)";
    if (p->m_total < 0) return "m_total must be >= 0 (0: no depletion)";
    if (p->motor_cfl < 0) return "motor_cfl must be >= 0 (0: no sub-cycling)";
    if (p->rc < 0) return "rc must be >= 0 (0: anchor-marginal model)";
    if (p->rc > 0 && !(p->rc + 0.5 * p->L < 0.5 * p->lx && p->rc + 0.5 * p->L < 0.5 * p->ly))
        return "rc + L/2 must be below lx/2 and ly/2 (each anchor-filament pair has one offset)";
    if ((int64_t)p->nx * p->ny > ((int64_t)1 << 31)) return "nx * ny too large";
    return "";
}

std::string check_supported(const mmk_params *p) {
    if (p->ntheta > kMaxTheta) return "ntheta > 512 is not supported by the psi kernel";
    if (p->ns > kMaxS) return "ns > 512 is not supported by the motor kernel";
    if (plan_psi(p->nx, p->ny, p->ntheta, esize(*p), 2).lds_bytes > 64 * 1024)
        return "ntheta too large for the psi kernel's LDS tile at this precision";
    if (p->rc > 0) {
        const R0Plan rp = r0_plan_of(*p);
        if (rp.lmax > kR0MaxRun) return "runs of tracked cells longer than 32 (rc too large for ns)";
        if (rp.ncell > INT32_MAX || (double)rp.ncell * p->nx * p->ny > 9.0e18) return "too many tracked cells";
    }
    return "";
}

Layout make_layout(const mmk_params &p, int ckpt_every, int max_tape_steps) {
    Layout L{};
    const size_t e = esize(p);
    const bool r0 = p.rc > 0;
    const R0Plan rp = r0 ? r0_plan_of(p) : R0Plan{};
    const size_t np = (size_t)n_psi(p), nxy = (size_t)p.nx * p.ny;
    // M, or the tiled anchor-resolved state (M[tile][cell][64 vx]) or its anchor layout
    // (M[r0][C/4][nthr][4]), whichever is larger
    const R0Slots rs = r0 ? r0_slots_of(p, rp) : R0Slots{};
    size_t nm = r0 ? (size_t)r0_tiled_elems(rp.ncell, (int64_t)nxy, r0_vx(e, rp.lmax)) : (size_t)n_m(p);
    if (rs.ok) nm = std::max(nm, (size_t)rs.per_anchor() * nxy);
    const PsiLaunch pl = plan_psi(p.nx, p.ny, p.ntheta, e, 2);
    const WalkPlan wp = plan_walk(p.nx, p.ny, p.ntheta);
    L.psi_blocks = wp.ok && wp.blocks > pl.blocks ? wp.blocks : pl.blocks;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.M[0] = take(nm * e);
    L.M[1] = take(nm * e);
    L.psi[0] = take(np * e);
    L.psi[1] = take(np * e);
    L.m0 = take(np * e);
    // temporal blocking of the linear motor step: m0 of the first kMaxBlock - 1 micro-steps
    // of a block, and a third psi buffer so that a block of any length ends in the other one
    L.m0s = (p.m_total > 0 || r0) ? 0 : take((size_t)(kMaxBlock - 1) * np * e);
    L.psi_tmp = (p.m_total > 0 || r0) ? 0 : take(np * e);
    L.m1 = take(np * e);
    L.Dxy = r0 ? 0 : take(2 * nxy * e);
    {
        // motor force: partial windows and the spreading records per (pass, cell)
        const ForcePlan fpl = plan_force(p.nx, p.ny, p.ntheta, p.ns, p.lx, p.ly, p.L, e);
        const size_t nblk = (size_t)fpl.npass * ((p.ns + fpl.chunk - 1) / fpl.chunk);
        L.fpart = take(fpl.part_elems * sizeof(double));
        L.fblk = take(nblk * kForceBlock * sizeof(uint32_t));
        L.fexy = take(2 * (size_t)fpl.npass * sizeof(int));
        L.fcs = take(2 * (size_t)fpl.npass * sizeof(double));
    }
    if (r0) {
        // the anchor-marginal field that the motor force spreads
        L.Mmarg = take((size_t)n_m(p) * e);
        // run totals, coarse partial rows, per-anchor clamp factor and pool, run table
        L.q0 = take((size_t)rp.nseg * nxy * e);
        L.r0part = take((size_t)4 * r0_coarse_split((int64_t)nxy, rp.nseg, e) * nxy * sizeof(double));
        L.r0scale = take(nxy * e);
        L.r0pool = take(nxy * e);
        L.r0seg = take((size_t)rp.nseg * sizeof(R0Seg));
        L.r0start = take(((size_t)p.ntheta + 1) * sizeof(int32_t));
        L.psiT = take(np * e);
        if (rs.ok) {
            L.q01 = take((size_t)2 * rp.nseg * ((nxy + 15) / 16 * 16) * e);  // tiles of 16 anchors
            L.r0slot = take(rs.slot_tab.size() * sizeof(int32_t));
            L.r0cpos = take(rs.cell_pos.size() * sizeof(int32_t));
        }
    }
    L.u = take(2 * nxy * e);
    L.G = take(4 * nxy * e);
    L.stress = take(3 * nxy * e);
    L.mom = take(7 * nxy * e);
    L.tab = take(TAB_N * (size_t)p.ntheta * e);
    L.partials = take((size_t)L.psi_blocks * 4 * sizeof(double));
    L.sums = take(4 * sizeof(double));
    off = tape_layout(&L.tape, off, nm, np, nxy, e, ckpt_every, max_tape_steps);
    L.total = off;
    return L;
}

}  // namespace

struct mmk_ctx {
    mmk_params p{};
    size_t esz = 8;
    hipStream_t stream = nullptr;
    int device = 0;
    char *ws = nullptr;
    Layout L{};
    PsiLaunch pl{}, pl_rev{};
    int cur = 0;    // index of the current M / psi buffers
    // implementation options (mmk_set_option), and what they select
    int opt[8] = {1, 0, 1, 0, 0, -1, 0, 1};
    // ntheta = 64, 128: the psi step runs as the LDS-free walking kernel (by default in FP32,
    // and in FP64 where nx allows the ring of register sets; apply_options decides)
    WalkPlan wp{};
    bool walk = false;
    bool block = false;  // temporal blocking of the linear motor step
    // the motor tiling of every untaped launch of this context: wide (32 bytes a lane) when the
    // launches carry several micro-steps or sub-steps per load; fixed per context so that
    // every launch sums the s-moments in the same order
    bool wide = false;
    // depletion with sub-cycling: every sub-step of a micro-step in one launch, one block per
    // (x, y) point, where the tiling allows it
    bool depl_fused = true;
    bool have_state = false, have_fluid = false, have_out = false;
    // The global sums (mass, sum sigma) reduce the FP64 block partials that the output psi launch
    // of the last call wrote; they are reduced when mmk_get_sums asks for them (sums_pending),
    // over sums_blocks rows (the psi kernel of that launch).
    bool sums_pending = false;
    int sums_blocks = 0;
    std::string err;
    bool prof = false;
    int prof_every[kProfIds] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1};  // time every n-th launch of each id (0: none)
    int64_t seen[kProfIds] = {};
    std::vector<hipEvent_t> ev[kProfIds];  // start/stop pairs
    int nev[kProfIds] = {};
    TapeState tape;
    // mmk_step_graph: captured K-step sequences by (K, dt, starting buffer), replayed on stream
    struct Graph {
        int K = 0, cur_in = 0, cur_out = 0;
        bool anch_in = false, anch_out = false;  // layout of the anchor-resolved state before and after
        bool q_pairs_in = false, q_pairs_out = false;  // which run totals are current before and after
        int sums_blocks = 0;  // partial rows the graph's output psi launch writes
        double dt = 0;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    hipStream_t capture_stream = nullptr;
    std::vector<double> host_tab64;  // host copies of the angle tables (outlive the async copy)
    std::vector<float> host_tab32;
    R0Plan r0;          // anchor-resolved model: tracked cells and runs (rc > 0)
    // One anchor per block (depleted sub-cycling in one pass): its slots, and whether the current
    // M buffer holds the anchor layout (set by those steps; the tiled layout is restored, into the
    // current buffer, by whatever needs it: the other steps, get_force).
    R0Slots r0s;
    bool r0_anch = false;
    bool q_pairs = false;  // the current run totals are the one-pass kernel's (q0, q1) pairs
    ForcePlan fplan;    // motor-force spreading geometry
    ForceRecords frec;  // host copy of the force spreading records
    std::vector<uint32_t> host_fblk;
    bool frec_ok = false;

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    void *vat(size_t off) const { return ws + off; }
};

// elements of the motor state: M [nx][ny][nth][ns], or Mb [ncell][nx][ny] when rc > 0 (the
// caller's layout; the context holds it tiled, r0_tiled_elems)
static int64_t n_state(const mmk_ctx *c) {
    return c->p.rc > 0 ? c->r0.ncell * (int64_t)c->p.nx * c->p.ny : n_m(c->p);
}
static int64_t n_state_held(const mmk_ctx *c) {
    return c->p.rc > 0 ? r0_tiled_elems(c->r0.ncell, (int64_t)c->p.nx * c->p.ny, r0_vx(c->esz, c->r0.lmax))
                       : n_m(c->p);
}

static mmk_status fail(mmk_ctx *c, mmk_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_create_error = buf;
    return st;
}

static mmk_status hipfail(mmk_ctx *c, hipError_t e, const char *what) {
    return fail(c, MMK_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(ctx, call, what)                       \
    do {                                              \
        hipError_t _e = (call);                       \
        if (_e != hipSuccess) return hipfail(ctx, _e, what); \
    } while (0)

// ---- profiling: event pairs around launches ---------------------------------------------
static hipError_t prof_begin_on(mmk_ctx *c, int id, int *slot, hipStream_t s) {
    *slot = -1;
    if (!c->prof || c->nev[id] >= kProfMax || c->prof_every[id] == 0) return hipSuccess;
    if (c->seen[id]++ % c->prof_every[id] != 0) return hipSuccess;
    int i = c->nev[id];
    while ((int)c->ev[id].size() < 2 * (i + 1)) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        c->ev[id].push_back(e);
    }
    *slot = i;
    return hipEventRecord(c->ev[id][2 * i], s);
}
static hipError_t prof_end_on(mmk_ctx *c, int id, int slot, hipStream_t s) {
    if (slot < 0) return hipSuccess;
    c->nev[id] = slot + 1;
    return hipEventRecord(c->ev[id][2 * slot + 1], s);
}
static hipError_t prof_begin(mmk_ctx *c, int id, int *slot) { return prof_begin_on(c, id, slot, c->stream); }
static hipError_t prof_end(mmk_ctx *c, int id, int slot) { return prof_end_on(c, id, slot, c->stream); }

// Drops the captured step graphs (their launches carry the options and buffers of the time
// they were captured).
static void drop_graphs(mmk_ctx *c) {
    for (auto &g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

// What the options select (mmk_set_option); called at create and after every change.
static void apply_options(mmk_ctx *c) {
    const mmk_params &p = c->p;
    const int psik = c->opt[MMK_OPT_PSI_KERNEL];
    // ring of register sets in the walk: 8 pencils at ntheta = 64, 4 at 128 (register space),
    // where the x extent is a multiple of the walk length
    const int depth = c->opt[MMK_OPT_PSI_DEPTH];
    const bool ring_ok = c->wp.ok && p.nx % c->wp.ti == 0;
    c->wp.depth = !ring_ok || depth == 2 ? 0 : depth == 0 ? (c->wp.kpl == 1 ? 8 : 4) : depth;
    // the walking kernel by default in FP32, and in FP64 where the ring applies (with two sets
    // the FP64 walk is slower than the LDS-tiled kernel)
    c->walk = c->wp.ok && (psik == 0 ? (c->esz == 4 || c->wp.depth > 0) : psik == 2);
    c->block = p.m_total == 0 && p.rc == 0 && c->opt[MMK_OPT_MOTOR_BLOCK] != 0;
    c->wide = c->block || (p.motor_cfl > 0 && p.m_total == 0);
    c->depl_fused = c->opt[MMK_OPT_DEPL_FUSED] != 0;
}

// Motor constants of one launch with the context's tiling options.
template <typename T>
static MotorConst<T> motor_cst(const mmk_ctx *c, double dt, bool wide) {
    MotorConst<T> mc = motor_const<T>(c->p, dt);
    mc.wide = wide ? 1 : 0;
    mc.lanes = c->opt[MMK_OPT_MOTOR_LANES];
    mc.chunks = c->opt[MMK_OPT_MOTOR_CHUNKS];
    mc.nt = c->opt[MMK_OPT_MOTOR_NT];
    return mc;
}

// ---- typed step ---------------------------------------------------------------------------
template <typename T>
static mmk_status motor_half(mmk_ctx *c, const T *M_in, T *M_out, T *m0, T *m1, double dt, hipStream_t s) {
    const mmk_params &p = c->p;
    int slot;
    HIPCHK(c, prof_begin_on(c, 0, &slot, s), "hipEventRecord");
    const T *Dxy = p.m_total > 0 ? c->at<T>(c->L.Dxy) : nullptr;
    const MotorConst<T> mc = motor_cst<T>(c, dt, c->wide && !c->tape.active);
    HIPCHK(c, launch_motor_step<T>(M_in, M_out, m0, m1, n_psi(p), p.ns, p.limiter, mc, Dxy, s), "motor step launch");
    HIPCHK(c, prof_end_on(c, 0, slot, s), "hipEventRecord");
    return MMK_OK;
}

template <typename T>
static mmk_status psi_half(mmk_ctx *c, const T *psi_in, T *psi_out, const T *m0, const T *m1, const T *u,
                           const T *G, double dt, bool out, hipStream_t s) {
    int slot;
    HIPCHK(c, prof_begin_on(c, 1, &slot, s), "hipEventRecord");
    T *stress = out ? c->at<T>(c->L.stress) : nullptr, *mom = out ? c->at<T>(c->L.mom) : nullptr;
    double *part = out ? c->at<double>(c->L.partials) : nullptr;
    // depletion factors of the new state (anchor-marginal model)
    T *Dxy = c->p.m_total > 0 && c->p.rc == 0 ? c->at<T>(c->L.Dxy) : nullptr;
    if (c->walk)
        HIPCHK(c, launch_psi_walk<T>(psi_in, psi_out, m0, m1, u, G, c->at<T>(c->L.tab), stress, mom, part, Dxy,
                                     psi_const<T>(c->p, dt), c->wp, s),
               "psi step launch");
    else
        HIPCHK(c, launch_psi_step<T>(psi_in, psi_out, m0, m1, u, G, c->at<T>(c->L.tab), stress, mom, part, Dxy,
                                     psi_const<T>(c->p, dt), c->pl, s),
               "psi step launch");
    HIPCHK(c, prof_end_on(c, 1, slot, s), "hipEventRecord");
    return MMK_OK;
}

// One micro-step from (M_in, psi_in) to (M_out, psi_out) on the context's stream.  With
// out = true also the stress, moments and the block partials of the global sums.
template <typename T>
static mmk_status micro_step(mmk_ctx *c, const T *M_in, T *M_out, const T *psi_in, T *psi_out, T *m0,
                             const T *u, const T *G, double dt, bool out) {
    T *m1 = out ? c->at<T>(c->L.m1) : nullptr;
    const mmk_params &p = c->p;
    const int nsub = (p.m_total > 0 && p.motor_cfl > 0) ? motor_substeps(p, dt) : 1;
    if (nsub > 1 && c->depl_fused && depl_sub_supported(c->esz, p.ntheta, p.ns, (int64_t)p.nx * p.ny)) {
        // depletion with sub-cycling (Alg. 2's inner loop) in one launch: each block re-forms the
        // clamp factor and the pool of its point before every sub-step, from psi of this step's
        // start and its columns held in registers
        int slot;
        HIPCHK(c, prof_begin(c, 0, &slot), "hipEventRecord");
        HIPCHK(c, launch_motor_depl_sub<T>(M_in, M_out, m0, m1, psi_in, (int64_t)p.nx * p.ny, p.ntheta, p.ns,
                                           p.limiter, motor_const<T>(p, dt), kTwoPi / p.ntheta, p.m_total, c->stream),
               "depleted sub-cycling launch");
        HIPCHK(c, prof_end(c, 0, slot), "hipEventRecord");
    } else if (nsub > 1) {
        // depletion with sub-cycling (Alg. 2's inner loop): n launches of one sub-step dt/n, each
        // with the clamp factors and pools of the current sub-state (the first from the psi
        // step before; then from psi of this step's start and the new m0).  The two M buffers
        // alternate (this path runs untaped: M_in, the context's own buffer, is not needed
        // after the step); an even n ends in M_in and is copied over.
        T *bufs[2] = {const_cast<T *>(M_in), M_out};
        T *Dxy = c->at<T>(c->L.Dxy);
        const int64_t np = n_psi(p), nxy = (int64_t)p.nx * p.ny;
        MotorConst<T> mc = motor_cst<T>(c, dt, false);  // dt / n per launch
        mc.nsub = 1;
        for (int q = 0; q < nsub; ++q) {
            if (q > 0)
                HIPCHK(c, launch_depletion_m0<T>(psi_in, m0, Dxy, nxy, p.ntheta, (T)(kTwoPi / p.ntheta), (T)p.m_total,
                                                 c->stream),
                       "depletion factors launch");
            int slot;
            HIPCHK(c, prof_begin(c, 0, &slot), "hipEventRecord");
            HIPCHK(c, launch_motor_step<T>(bufs[q % 2], bufs[(q + 1) % 2], m0, q + 1 == nsub ? m1 : nullptr, np, p.ns,
                                           p.limiter, mc, Dxy, c->stream),
                   "motor step launch");
            HIPCHK(c, prof_end(c, 0, slot), "hipEventRecord");
        }
        if (nsub % 2 == 0)
            HIPCHK(c, hipMemcpyAsync(M_out, M_in, (size_t)n_m(p) * c->esz, hipMemcpyDeviceToDevice, c->stream),
                   "copy of M");
    } else {
        mmk_status st = motor_half<T>(c, M_in, M_out, m0, m1, dt, c->stream);
        if (st != MMK_OK) return st;
    }
    return psi_half<T>(c, psi_in, psi_out, m0, m1, u, G, dt, out, c->stream);
}

template <typename T>
static mmk_status global_sums(mmk_ctx *c) {
    const mmk_params &p = c->p;
    const double dx = p.lx / p.nx, dy = p.ly / p.ny, dth = kTwoPi / p.ntheta;
    int slot;
    HIPCHK(c, prof_begin(c, 2, &slot), "hipEventRecord");
    HIPCHK(c, launch_reduce_partials(c->at<double>(c->L.partials), c->sums_blocks,
                                     c->at<double>(c->L.sums),
                                     dx * dy * dth, dx * dy, c->stream),
           "global sums launch");
    HIPCHK(c, prof_end(c, 2, slot), "hipEventRecord");
    return MMK_OK;
}

// Sequential order: motor step then psi step, both on the context's stream (taped runs).
template <typename T>
static mmk_status run_steps_serial(mmk_ctx *c, int K, double dt) {
    for (int n = 0; n < K; ++n) {
        const bool last = (n == K - 1);
        const int a = c->cur, b = 1 - c->cur;
        mmk_status st = tape_before_step(c, &c->tape, dt);
        if (st != MMK_OK) return st;
        st = micro_step<T>(c, c->at<T>(c->L.M[a]), c->at<T>(c->L.M[b]), c->at<T>(c->L.psi[a]),
                           c->at<T>(c->L.psi[b]), c->at<T>(c->L.m0), c->at<T>(c->L.u), c->at<T>(c->L.G),
                           dt, last);
        if (st != MMK_OK) return st;
        c->cur = b;
        st = tape_after_step(c, &c->tape);
        if (st != MMK_OK) return st;
    }
    return MMK_OK;
}

// Temporal blocking of the linear motor step (m_total = 0, no tape): M does not depend on psi,
// so one motor launch advances M through a block of up to kMaxBlock micro-steps, keeping each
// column in registers and leaving m0 of every micro-step; then the block's psi steps run, each
// with the m0 of its own micro-step.  Every micro-step is computed exactly as in the serial
// order (the same bits); M is read and written once per block instead of once per step.
template <typename T>
static mmk_status run_steps_blocked(mmk_ctx *c, int K, double dt) {
    const mmk_params &p = c->p;
    const int64_t np = n_psi(p);
    T *m0 = c->at<T>(c->L.m0), *m0s = c->at<T>(c->L.m0s), *m1 = c->at<T>(c->L.m1);
    const T *u = c->at<T>(c->L.u), *G = c->at<T>(c->L.G);
    for (int done = 0; done < K;) {
        const int nb = std::min(kMaxBlock, K - done);
        const bool out = done + nb == K;  // the call's last micro-step, with the outputs
        const int a = c->cur, b = 1 - c->cur;
        MotorConst<T> mc = motor_cst<T>(c, dt, c->wide);
        mc.nstep = nb;
        mc.m0_steps = m0s;
        int slot;
        HIPCHK(c, prof_begin_on(c, 0, &slot, c->stream), "hipEventRecord");
        HIPCHK(c, launch_motor_step<T>(c->at<T>(c->L.M[a]), c->at<T>(c->L.M[b]), m0, out ? m1 : nullptr, np, p.ns,
                                       p.limiter, mc, nullptr, c->stream),
               "motor step launch");
        HIPCHK(c, prof_end_on(c, 0, slot, c->stream), "hipEventRecord");
        // psi from buffer a to buffer b: the steps alternate between b and the third buffer,
        // counted back from the last one, which writes b
        const T *src = c->at<T>(c->L.psi[a]);
        for (int t = 0; t < nb; ++t) {
            T *dst = ((nb - 1 - t) % 2 == 0) ? c->at<T>(c->L.psi[b]) : c->at<T>(c->L.psi_tmp);
            const T *m0t = t + 1 < nb ? m0s + (int64_t)t * np : m0;
            mmk_status st = psi_half<T>(c, src, dst, m0t, m1, u, G, dt, out && t + 1 == nb, c->stream);
            if (st != MMK_OK) return st;
            src = dst;
        }
        c->cur = b;
        done += nb;
    }
    return MMK_OK;
}

// ---- anchor-resolved model -----------------------------------------------------------------
template <typename T>
static R0Const<T> r0_const(const mmk_params &p, double dt, int advance) {
    const double ds = p.L / p.ns;
    R0Const<T> c;
    c.k_on = (T)p.k_on;
    c.k_off = (T)p.k_off;
    c.nv_ds = (T)(-p.v0 / ds);
    c.dt = (T)dt;
    c.half_dt = (T)(0.5 * dt);
    c.ds = ds;
    c.ds2 = ds * ds;
    c.dA = (p.lx / p.nx) * (p.ly / p.ny);
    c.half_ns = 0.5 * p.ns;
    c.nx = p.nx;
    c.ny = p.ny;
    c.nth = p.ntheta;
    c.nxy = (int64_t)p.nx * p.ny;
    c.ncell = 0;
    c.vx = 1;
    c.advance = advance;
    c.nsub = 1;
    return c;
}

template <typename T>
static R0Const<T> r0_cst(const mmk_ctx *c, double dt, int advance) {
    R0Const<T> k = r0_const<T>(c->p, dt, advance);
    k.ncell = c->r0.ncell;
    k.vx = r0_vx(sizeof(T), c->r0.lmax);
    return k;
}

template <typename T>
static R0Const<T> r0_with_nsub(R0Const<T> k, int nsub) {
    k.nsub = nsub;
    return k;
}

// nsub motor steps of dt of every run (advance = 0: only the run totals and marginals of the
// current state).
template <typename T>
static mmk_status r0_motor(mmk_ctx *c, const T *M_in, T *M_out, double dt, int advance, bool clamp, int nsub = 1) {
    const mmk_params &p = c->p;
    int slot;
    HIPCHK(c, prof_begin(c, 6, &slot), "hipEventRecord");
    HIPCHK(c, launch_r0_motor<T>(M_in, M_out, c->at<T>(c->L.q0), c->at<T>(c->L.m0), c->at<T>(c->L.m1),
                                 c->at<R0Seg>(c->L.r0seg), c->at<int32_t>(c->L.r0start),
                                 clamp ? c->at<T>(c->L.r0scale) : nullptr, clamp ? c->at<T>(c->L.r0pool) : nullptr,
                                 r0_with_nsub(r0_cst<T>(c, dt, advance), nsub), c->r0.lmax, p.limiter, c->stream),
           "anchor-resolved motor launch");
    HIPCHK(c, prof_end(c, 6, slot), "hipEventRecord");
    c->q_pairs = false;
    return MMK_OK;
}

// Coarse density of every anchor of the current state; with clamp, the factor and pool of the
// next motor step; coarse_out / free_out (may be NULL) in the field precision.
template <typename T>
static mmk_status r0_anchors(mmk_ctx *c, bool clamp, T *coarse_out, T *free_out) {
    const mmk_params &p = c->p;
    int slot;
    HIPCHK(c, prof_begin(c, 7, &slot), "hipEventRecord");
    HIPCHK(c, launch_r0_coarse<T>(c->q_pairs ? c->at<T>(c->L.q01) : c->at<T>(c->L.q0), c->q_pairs,
                                  c->at<T>(c->L.psi[c->cur]), c->at<T>(c->L.psiT),
                                  c->at<R0Seg>(c->L.r0seg),
                                  c->at<double>(c->L.r0part), clamp ? c->at<T>(c->L.r0scale) : nullptr,
                                  clamp ? c->at<T>(c->L.r0pool) : nullptr, coarse_out, free_out,
                                  r0_cst<T>(c, 0.0, 0), c->r0.nseg, c->r0.nsplit, kTwoPi / p.ntheta, p.m_total,
                                  p.k_on, c->stream),
           "anchor coarse density launch");
    HIPCHK(c, prof_end(c, 7, slot), "hipEventRecord");
    return MMK_OK;
}

// The anchor-resolved state back in the tiled layout, in the current buffer (through the other
// one), if the one-pass steps left it in the anchor layout.
template <typename T>
static mmk_status r0_tiled(mmk_ctx *c) {
    if (!c->r0_anch) return MMK_OK;
    const int a = c->cur, b = 1 - c->cur;
    const int vx = r0_vx(sizeof(T), c->r0.lmax);
    HIPCHK(c, launch_r0_anchor_layout<T>(c->at<T>(c->L.M[a]), c->at<T>(c->L.M[b]), c->at<int32_t>(c->L.r0cpos),
                                         r0_cst<T>(c, 0.0, 0), vx, c->r0s.per_anchor(), c->r0s.nthr, false, c->stream),
           "anchor -> tiled layout of Mb");
    HIPCHK(c, hipMemcpyAsync(c->at<T>(c->L.M[a]), c->at<T>(c->L.M[b]), (size_t)n_state_held(c) * sizeof(T),
                             hipMemcpyDeviceToDevice, c->stream),
           "copy of Mb");
    c->r0_anch = false;
    return MMK_OK;
}

// One micro-step's nsub motor sub-steps of dt with the clamp re-formed before each, one anchor per
// block (anchor layout, M_in -> M_out, in place allowed), then m0, m1 from the run totals.
template <typename T>
static mmk_status r0_onepass(mmk_ctx *c, const T *M_in, T *M_out, double dt, int nsub) {
    const mmk_params &p = c->p;
    int slot;
    HIPCHK(c, prof_begin(c, 8, &slot), "hipEventRecord");
    HIPCHK(c, launch_r0_anchor<T>(M_in, M_out, c->at<T>(c->L.q01), c->at<int32_t>(c->L.r0slot),
                                  c->at<T>(c->L.psi[c->cur]), r0_cst<T>(c, dt, 1), c->r0.nseg,
                                  c->r0s.C, c->r0s.nthr, nsub, p.m_total, p.k_on, kTwoPi / p.ntheta, p.limiter,
                                  c->stream),
           "anchor-owned motor launch");
    HIPCHK(c, prof_end(c, 8, slot), "hipEventRecord");
    HIPCHK(c, prof_begin(c, 9, &slot), "hipEventRecord");
    HIPCHK(c, launch_r0_marg<T>(c->at<T>(c->L.q01), c->r0.nseg, c->at<R0Seg>(c->L.r0seg),
                                c->at<int32_t>(c->L.r0start), c->at<T>(c->L.m0), c->at<T>(c->L.m1),
                                r0_cst<T>(c, 0.0, 0), c->stream),
           "anchor marginals launch");
    HIPCHK(c, prof_end(c, 9, slot), "hipEventRecord");
    c->q_pairs = true;
    return MMK_OK;
}

// Each micro-step: n motor sub-steps of dt/n (motor_substeps; n = 1 without sub-cycling), then
// psi driven by the marginal m0.  With m_total > 0 the clamp is re-formed before every sub-step
// (psi of the step's start; Alg. 2 clamps inside its inner loop): where the tracked set fits one
// block (MMK_OPT_R0_ONEPASS), one launch holds each anchor's cells and runs all n sub-steps
// (anchor layout, converted to on the first such step); otherwise each sub-step is its own
// launch after the coarse density, clamp and pool of the current sub-state, alternating between
// the two M buffers (an even n ends in the first and is copied over).  Without depletion one
// launch takes all n sub-steps in registers.
template <typename T>
static mmk_status run_steps_r0(mmk_ctx *c, int K, double dt) {
    const bool depl = c->p.m_total > 0;
    const int nsub = motor_substeps(c->p, dt);
    const double h = dt / nsub;
    const bool onepass = depl && nsub > 1 && c->r0s.ok && c->opt[MMK_OPT_R0_ONEPASS] != 0;
    if (!onepass) {
        const mmk_status st = r0_tiled<T>(c);
        if (st != MMK_OK) return st;
    }
    const size_t mbytes = (size_t)n_state_held(c) * sizeof(T);
    for (int n = 0; n < K; ++n) {
        const int a = c->cur, b = 1 - c->cur;
        mmk_status st = MMK_OK;
        if (onepass) {
            const T *in = c->at<T>(c->L.M[a]);
            if (!c->r0_anch) {  // tiled -> anchor layout, into the other buffer; the step runs in place
                HIPCHK(c, launch_r0_anchor_layout<T>(in, c->at<T>(c->L.M[b]), c->at<int32_t>(c->L.r0cpos),
                                                     r0_cst<T>(c, 0.0, 0), r0_vx(sizeof(T), c->r0.lmax),
                                                     c->r0s.per_anchor(), c->r0s.nthr, true, c->stream),
                       "tiled -> anchor layout of Mb");
                in = c->at<T>(c->L.M[b]);
                c->r0_anch = true;
            }
            st = r0_onepass<T>(c, in, c->at<T>(c->L.M[b]), h, nsub);
        } else if (!depl) {
            st = r0_motor<T>(c, c->at<T>(c->L.M[a]), c->at<T>(c->L.M[b]), h, 1, false, nsub);
        } else {
            for (int q = 0; q < nsub && st == MMK_OK; ++q) {
                st = r0_anchors<T>(c, true, nullptr, nullptr);
                if (st == MMK_OK)
                    st = r0_motor<T>(c, c->at<T>(c->L.M[q % 2 ? b : a]), c->at<T>(c->L.M[q % 2 ? a : b]), h, 1, true);
            }
            if (st == MMK_OK && nsub % 2 == 0 && mbytes > 0)
                HIPCHK(c, hipMemcpyAsync(c->at<T>(c->L.M[b]), c->at<T>(c->L.M[a]), mbytes, hipMemcpyDeviceToDevice,
                                         c->stream),
                       "copy of M_b");
        }
        if (st == MMK_OK)
            st = psi_half<T>(c, c->at<T>(c->L.psi[a]), c->at<T>(c->L.psi[b]), c->at<T>(c->L.m0), c->at<T>(c->L.m1),
                             c->at<T>(c->L.u), c->at<T>(c->L.G), dt, n == K - 1, c->stream);
        if (st != MMK_OK) return st;
        c->cur = b;
    }
    return MMK_OK;
}

template <typename T>
static mmk_status run_steps(mmk_ctx *c, int K, double dt) {
    const bool blocked = c->block && c->p.m_total == 0 && !c->tape.active;
    mmk_status st = c->p.rc > 0 ? run_steps_r0<T>(c, K, dt)
                    : blocked   ? run_steps_blocked<T>(c, K, dt)
                                : run_steps_serial<T>(c, K, dt);
    if (st != MMK_OK) return st;
    if (K > 0) {
        c->have_out = true;
        c->sums_pending = true;
        c->sums_blocks = c->walk ? c->wp.blocks : c->pl.blocks;
    }
    return MMK_OK;
}

// ---- internal accessors used by the tape ---------------------------------------------------
namespace mmk {
const mmk_params &ctx_params(const mmk_ctx *c) { return c->p; }
hipStream_t ctx_stream(const mmk_ctx *c) { return c->stream; }
char *ctx_ws(const mmk_ctx *c) { return c->ws; }
size_t ctx_esz(const mmk_ctx *c) { return c->esz; }
const TapeLayout &ctx_tape_layout(const mmk_ctx *c) { return c->L.tape; }
void *ctx_cur_M(const mmk_ctx *c) { return c->ws + c->L.M[c->cur]; }
void *ctx_cur_psi(const mmk_ctx *c) { return c->ws + c->L.psi[c->cur]; }
void *ctx_fluid_u(const mmk_ctx *c) { return c->ws + c->L.u; }
void *ctx_fluid_G(const mmk_ctx *c) { return c->ws + c->L.G; }
void *ctx_m0(const mmk_ctx *c) { return c->ws + c->L.m0; }
void *ctx_m1(const mmk_ctx *c) { return c->ws + c->L.m1; }
void *ctx_tab(const mmk_ctx *c) { return c->ws + c->L.tab; }
const PsiLaunch &ctx_psi_launch(const mmk_ctx *c) { return c->pl; }
const PsiLaunch &ctx_psi_launch_rev(const mmk_ctx *c) { return c->pl_rev; }
bool ctx_have_out(const mmk_ctx *c) { return c->have_out; }
mmk_status ctx_fail(mmk_ctx *c, mmk_status st, const char *msg) { return fail(c, st, "%s", msg); }
mmk_status ctx_hipfail(mmk_ctx *c, hipError_t e, const char *what) { return hipfail(c, e, what); }
hipError_t ctx_prof_begin(mmk_ctx *c, int id, int *slot) { return prof_begin(c, id, slot); }
hipError_t ctx_prof_end(mmk_ctx *c, int id, int slot) { return prof_end(c, id, slot); }
template <typename T>
mmk_status ctx_forward_step(mmk_ctx *c, const T *M_in, T *M_out, const T *psi_in, T *psi_out, T *m0,
                            const T *u, const T *G, double dt) {
    return micro_step<T>(c, M_in, M_out, psi_in, psi_out, m0, u, G, dt, false);
}
template mmk_status ctx_forward_step<float>(mmk_ctx *, const float *, float *, const float *, float *, float *,
                                            const float *, const float *, double);
template mmk_status ctx_forward_step<double>(mmk_ctx *, const double *, double *, const double *, double *,
                                             double *, const double *, const double *, double);
}  // namespace mmk

// ---- C-ABI ----------------------------------------------------------------------------------
extern "C" {

size_t mmk_workspace_bytes(const mmk_params *p, int32_t ckpt_every, int32_t max_tape_steps) {
    std::string m = check_params(p);
    if (m.empty()) m = check_supported(p);
    if (m.empty() && ckpt_every < 0) m = "ckpt_every must be >= 0";
    if (m.empty() && ckpt_every > 0 && max_tape_steps < 0) m = "max_tape_steps must be >= 0";
    if (!m.empty()) {
        g_create_error = m;
        return 0;
    }
    return make_layout(*p, ckpt_every, ckpt_every > 0 ? max_tape_steps : 0).total;
}

mmk_status mmk_create(const mmk_params *p, void *workspace, size_t ws_bytes, void *hip_stream,
                      int32_t ckpt_every, int32_t max_tape_steps, mmk_ctx **out) {
    if (!out) return fail(nullptr, MMK_ERR_ARG, "out is NULL");
    *out = nullptr;
    std::string m = check_params(p);
    if (!m.empty()) return fail(nullptr, MMK_ERR_ARG, "%s", m.c_str());
    m = check_supported(p);
    if (!m.empty()) return fail(nullptr, MMK_ERR_UNSUPPORTED, "%s", m.c_str());
    if (ckpt_every < 0 || (ckpt_every > 0 && max_tape_steps < 0))
        return fail(nullptr, MMK_ERR_ARG, "ckpt_every and max_tape_steps must be >= 0");
    if (ckpt_every > 0 && p->rc > 0)
        return fail(nullptr, MMK_ERR_UNSUPPORTED, "the adjoint tape covers the anchor-marginal model only (rc = 0)");
    if (ckpt_every > 0 && plan_psi(p->nx, p->ny, p->ntheta, esize(*p), 3).lds_bytes > 64 * 1024)
        return fail(nullptr, MMK_ERR_UNSUPPORTED, "ntheta too large for the reverse psi kernel at this precision");
    if (!workspace) return fail(nullptr, MMK_ERR_ARG, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(nullptr, MMK_ERR_ARG, "workspace must be 256-byte aligned");
    const Layout L = make_layout(*p, ckpt_every, ckpt_every > 0 ? max_tape_steps : 0);
    if (ws_bytes < L.total)
        return fail(nullptr, MMK_ERR_NOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    mmk_ctx *c = new mmk_ctx();
    c->p = *p;
    c->esz = esize(*p);
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char *)workspace;
    c->L = L;
    c->pl = plan_psi(p->nx, p->ny, p->ntheta, c->esz, 2);
    c->pl_rev = plan_psi(p->nx, p->ny, p->ntheta, c->esz, 3);
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return hipfail(nullptr, e, "hipGetDevice");
    }
    // angle tables, computed on the host in FP64 and rounded to the field precision
    const int nth = p->ntheta;
    const double dth = kTwoPi / nth;
    std::vector<double> t((size_t)TAB_N * nth);
    for (int k = 0; k < nth; ++k) {
        const double th = k * dth, tf = (k + 0.5) * dth;
        const double co = std::cos(th), si = std::sin(th);
        t[TAB_C * nth + k] = co;
        t[TAB_S * nth + k] = si;
        t[TAB_CH * nth + k] = std::cos(tf);
        t[TAB_SH * nth + k] = std::sin(tf);
        t[TAB_H1 * nth + k] = 0.5 * std::cos(2.0 * th);
        t[TAB_H2 * nth + k] = 0.5 * std::sin(2.0 * th);
        t[TAB_CC * nth + k] = co * co;
        t[TAB_CS * nth + k] = co * si;
        t[TAB_SS * nth + k] = si * si;
    }
    c->host_tab64 = t;
    if (c->esz == 4) {
        c->host_tab32.assign(t.begin(), t.end());
        e = hipMemcpyAsync(c->ws + L.tab, c->host_tab32.data(), t.size() * 4, hipMemcpyHostToDevice, c->stream);
    } else {
        e = hipMemcpyAsync(c->ws + L.tab, c->host_tab64.data(), t.size() * 8, hipMemcpyHostToDevice, c->stream);
    }
    // spreading records of the motor force (needed only by mmk_get_force; anchor-marginal model)
    c->fplan = plan_force(p->nx, p->ny, nth, p->ns, p->lx, p->ly, p->L, c->esz);
    ForceRecords &fr = c->frec;
    c->frec_ok = force_records(nth, p->ns, p->lx, p->ly, p->L, p->nx, p->ny, c->fplan, &fr);
    if (p->rc > 0) {  // tracked cells and runs of the anchor-resolved model
        c->r0 = r0_plan_of(*p);
        c->r0.nsplit = r0_coarse_split((int64_t)p->nx * p->ny, c->r0.nseg, c->esz);
        if (e == hipSuccess && c->r0.nseg > 0)
            e = hipMemcpyAsync(c->ws + L.r0seg, c->r0.seg.data(), c->r0.seg.size() * sizeof(R0Seg),
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ws + L.r0start, c->r0.seg_start.data(), c->r0.seg_start.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, c->stream);
        c->r0s = r0_slots_of(*p, c->r0);
        if (e == hipSuccess && c->r0s.ok)
            e = hipMemcpyAsync(c->ws + L.r0slot, c->r0s.slot_tab.data(), c->r0s.slot_tab.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && c->r0s.ok)
            e = hipMemcpyAsync(c->ws + L.r0cpos, c->r0s.cell_pos.data(), c->r0s.cell_pos.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, c->stream);
    }
    if (c->frec_ok) {
        auto up = [&](size_t off, const void *src, size_t bytes) {
            if (e == hipSuccess) e = hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
        };
        force_record_blocks(fr, c->fplan, c->esz, &c->host_fblk);
        up(L.fblk, c->host_fblk.data(), c->host_fblk.size() * sizeof(uint32_t));
        up(L.fexy, fr.exy.data(), fr.exy.size() * sizeof(int));
        up(L.fcs, fr.cs.data(), fr.cs.size() * sizeof(double));
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return hipfail(nullptr, e, "copy of angle tables");
    }
    tape_init(&c->tape, ckpt_every, ckpt_every > 0 ? max_tape_steps : 0);
    c->wp = plan_walk(p->nx, p->ny, p->ntheta);
    apply_options(c);
    *out = c;
    return MMK_OK;
}

mmk_status mmk_destroy(mmk_ctx *c) {
    if (!c) return MMK_ERR_ARG;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (int i = 0; i < kProfIds; ++i)
        for (hipEvent_t e : c->ev[i]) (void)hipEventDestroy(e);
    delete c;
    return MMK_OK;
}

mmk_status mmk_set_params(mmk_ctx *c, double k_on, double k_off, double v0) {
    if (!c) return MMK_ERR_ARG;
    if (!std::isfinite(k_on) || !std::isfinite(k_off) || !std::isfinite(v0))
        return fail(c, MMK_ERR_ARG, "non-finite rate");
    if (v0 < 0) return fail(c, MMK_ERR_ARG, "v0 must be >= 0");
    if (c->tape.active && c->tape.steps > 0)
        return fail(c, MMK_ERR_STATE, "parameters cannot change inside a taped run");
    c->p.k_on = k_on;
    c->p.k_off = k_off;
    c->p.v0 = v0;
    drop_graphs(c);
    return MMK_OK;
}

mmk_status mmk_set_option(mmk_ctx *c, int32_t option, int32_t value) {
    if (!c) return MMK_ERR_ARG;
    bool ok;
    switch (option) {
        case MMK_OPT_MOTOR_BLOCK:
        case MMK_OPT_DEPL_FUSED:
        case MMK_OPT_R0_ONEPASS: ok = value == 0 || value == 1; break;
        case MMK_OPT_PSI_KERNEL: ok = value >= 0 && value <= 2; break;
        case MMK_OPT_MOTOR_LANES: ok = value == 0 || (value >= 2 && value <= 64 && (value & (value - 1)) == 0); break;
        case MMK_OPT_MOTOR_CHUNKS: ok = value == 0 || value == 1 || value == 2 || value == 4; break;
        case MMK_OPT_MOTOR_NT: ok = value >= -1 && value <= 2; break;
        case MMK_OPT_PSI_DEPTH: ok = value == 0 || value == 2 || value == 4 || value == 8; break;
        default: return fail(c, MMK_ERR_ARG, "unknown option %d", option);
    }
    if (!ok) return fail(c, MMK_ERR_ARG, "value %d out of range for option %d", value, option);
    c->opt[option] = value;
    apply_options(c);
    drop_graphs(c);
    return MMK_OK;
}

mmk_status mmk_set_state(mmk_ctx *c, const void *psi, const void *M) {
    if (!c) return MMK_ERR_ARG;
    if (!psi) return fail(c, MMK_ERR_ARG, "psi is NULL");
    if (c->tape.active) return fail(c, MMK_ERR_STATE, "set_state during a taped run");
    const int64_t nme = n_state(c), held = n_state_held(c);
    const size_t np = (size_t)n_psi(c->p) * c->esz, nm = (size_t)nme * c->esz;
    const int64_t nxy = (int64_t)c->p.nx * c->p.ny;
    const int vx = r0_vx(c->esz, c->r0.lmax);
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.psi[c->cur], psi, np, hipMemcpyDeviceToDevice, c->stream),
           "copy of psi");
    c->r0_anch = false;
    if (M && nm > 0 && c->p.rc > 0) {  // caller layout -> tiled
        HIPCHK(c, c->esz == 4 ? launch_r0_layout<float>((const float *)M, c->at<float>(c->L.M[c->cur]), c->r0.ncell, nxy, vx, true, c->stream)
                              : launch_r0_layout<double>((const double *)M, c->at<double>(c->L.M[c->cur]), c->r0.ncell, nxy, vx, true, c->stream),
               "layout of Mb");
    } else if (M && nm > 0) {
        HIPCHK(c, hipMemcpyAsync(c->ws + c->L.M[c->cur], M, nm, hipMemcpyDeviceToDevice, c->stream), "copy of M");
    } else if (c->esz == 4) {
        HIPCHK(c, launch_zero<float>(c->at<float>(c->L.M[c->cur]), held, c->stream), "zero M");
    } else {
        HIPCHK(c, launch_zero<double>(c->at<double>(c->L.M[c->cur]), held, c->stream), "zero M");
    }
    if (c->p.rc > 0) {  // run totals and anchor marginals of the new state, for the first step
        mmk_status st = c->esz == 4 ? r0_motor<float>(c, c->at<float>(c->L.M[c->cur]), c->at<float>(c->L.M[c->cur]), 0.0, 0, false)
                                    : r0_motor<double>(c, c->at<double>(c->L.M[c->cur]), c->at<double>(c->L.M[c->cur]), 0.0, 0, false);
        if (st != MMK_OK) return st;
    } else if (c->p.m_total > 0) {  // depletion factors of the new state, for the first step
        const double ds = c->p.L / c->p.ns, dth = kTwoPi / c->p.ntheta;
        const int64_t nxy = (int64_t)c->p.nx * c->p.ny;
        hipError_t e;
        if (c->esz == 4)
            e = launch_coarse_bound<float>(M ? c->at<float>(c->L.M[c->cur]) : nullptr, c->at<float>(c->L.psi[c->cur]),
                                           c->at<float>(c->L.Dxy), nxy, c->p.ntheta, c->p.ns, (float)ds, (float)dth,
                                           (float)c->p.m_total, c->stream);
        else
            e = launch_coarse_bound<double>(M ? c->at<double>(c->L.M[c->cur]) : nullptr,
                                            c->at<double>(c->L.psi[c->cur]), c->at<double>(c->L.Dxy), nxy,
                                            c->p.ntheta, c->p.ns, ds, dth, c->p.m_total, c->stream);
        HIPCHK(c, e, "coarse bound density launch");
    }
    c->have_state = true;
    c->have_out = false;
    return MMK_OK;
}

mmk_status mmk_set_fluid(mmk_ctx *c, const void *u, const void *gradu) {
    if (!c) return MMK_ERR_ARG;
    if (!u || !gradu) return fail(c, MMK_ERR_ARG, "u or gradu is NULL");
    const size_t nxy = (size_t)c->p.nx * c->p.ny * c->esz;
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.u, u, 2 * nxy, hipMemcpyDeviceToDevice, c->stream), "copy of u");
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.G, gradu, 4 * nxy, hipMemcpyDeviceToDevice, c->stream), "copy of gradu");
    c->have_fluid = true;
    return tape_on_fluid(c, &c->tape);
}

mmk_status mmk_step(mmk_ctx *c, int32_t K, double dt) {
    if (!c) return MMK_ERR_ARG;
    if (K < 0) return fail(c, MMK_ERR_ARG, "K must be >= 0");
    if (!std::isfinite(dt) || dt <= 0) return fail(c, MMK_ERR_ARG, "dt must be finite and > 0");
    if (!c->have_state) return fail(c, MMK_ERR_STATE, "mmk_step before mmk_set_state");
    if (!c->have_fluid) return fail(c, MMK_ERR_STATE, "mmk_step before mmk_set_fluid");
    if (K == 0) return MMK_OK;
    if (motor_substeps(c->p, dt) < 1)
        return fail(c, MMK_ERR_ARG, "dt (v0/ds + k_off) / motor_cfl needs more than %d motor sub-steps",
                    kMaxSubsteps);
    if (c->tape.active && c->tape.steps + K > c->tape.max_steps)
        return fail(c, MMK_ERR_ARG, "taped run would exceed max_tape_steps (%d)", c->tape.max_steps);
    return c->esz == 4 ? run_steps<float>(c, K, dt) : run_steps<double>(c, K, dt);
}

mmk_status mmk_step_graph(mmk_ctx *c, int32_t K, double dt) {
    if (!c) return MMK_ERR_ARG;
    if (K < 0) return fail(c, MMK_ERR_ARG, "K must be >= 0");
    if (!std::isfinite(dt) || dt <= 0) return fail(c, MMK_ERR_ARG, "dt must be finite and > 0");
    if (!c->have_state) return fail(c, MMK_ERR_STATE, "mmk_step_graph before mmk_set_state");
    if (!c->have_fluid) return fail(c, MMK_ERR_STATE, "mmk_step_graph before mmk_set_fluid");
    if (c->tape.active) return fail(c, MMK_ERR_STATE, "mmk_step_graph during a taped run (use mmk_step)");
    if (K == 0) return MMK_OK;
    if (motor_substeps(c->p, dt) < 1)
        return fail(c, MMK_ERR_ARG, "dt (v0/ds + k_off) / motor_cfl needs more than %d motor sub-steps",
                    kMaxSubsteps);
    mmk_ctx::Graph *g = nullptr;
    for (auto &x : c->graphs)
        if (x.K == K && x.dt == dt && x.cur_in == c->cur && x.anch_in == c->r0_anch && x.q_pairs_in == c->q_pairs)
            g = &x;
    if (!g) {
        if (c->graphs.size() >= 8) drop_graphs(c);
        if (!c->capture_stream)
            HIPCHK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
        // record the launches of mmk_step(K, dt) from this buffer into a graph: the same code
        // path enqueues them on a capturing stream of the library's own (nothing runs)
        mmk_ctx::Graph ng;
        ng.K = K;
        ng.dt = dt;
        ng.cur_in = c->cur;
        ng.anch_in = c->r0_anch;
        const bool qp = c->q_pairs;
        ng.q_pairs_in = qp;
        hipStream_t user = c->stream;
        const bool prof = c->prof, pending = c->sums_pending;
        const int blocks = c->sums_blocks;
        c->prof = false;
        c->stream = c->capture_stream;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        mmk_status st = MMK_OK;
        if (e == hipSuccess) st = c->esz == 4 ? run_steps<float>(c, K, dt) : run_steps<double>(c, K, dt);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(c->stream, &graph) : e;
        c->stream = user;
        c->prof = prof;
        ng.cur_out = c->cur;
        ng.anch_out = c->r0_anch;
        ng.q_pairs_out = c->q_pairs;
        c->q_pairs = qp;
        ng.sums_blocks = c->sums_blocks;
        c->cur = ng.cur_in;  // nothing has run yet
        c->r0_anch = ng.anch_in;
        c->sums_pending = pending;
        c->sums_blocks = blocks;
        if (e != hipSuccess) return hipfail(c, e, "hipStreamBeginCapture");
        if (st != MMK_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e2 != hipSuccess) return hipfail(c, e2, "hipStreamEndCapture");
        e = hipGraphInstantiate(&ng.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hipfail(c, e, "hipGraphInstantiate");
        c->graphs.push_back(ng);
        g = &c->graphs.back();
    }
    HIPCHK(c, hipGraphLaunch(g->exec, c->stream), "hipGraphLaunch");
    c->cur = g->cur_out;
    c->r0_anch = g->anch_out;
    c->q_pairs = g->q_pairs_out;
    c->have_out = true;
    c->sums_pending = true;
    c->sums_blocks = g->sums_blocks;
    return MMK_OK;
}

mmk_status mmk_get_state(mmk_ctx *c, void *psi, void *M) {
    if (!c) return MMK_ERR_ARG;
    if (!c->have_state) return fail(c, MMK_ERR_STATE, "no state set");
    if (psi)
        HIPCHK(c, hipMemcpyAsync(psi, c->ws + c->L.psi[c->cur], (size_t)n_psi(c->p) * c->esz,
                                 hipMemcpyDeviceToDevice, c->stream), "copy of psi");
    if (M && n_state(c) > 0 && c->p.rc > 0 && c->r0_anch) {  // anchor -> caller layout
        HIPCHK(c, c->esz == 4 ? launch_r0_anchor_layout<float>(c->at<float>(c->L.M[c->cur]), (float *)M,
                                                               c->at<int32_t>(c->L.r0cpos), r0_cst<float>(c, 0.0, 0),
                                                               0, c->r0s.per_anchor(), c->r0s.nthr, false, c->stream)
                              : launch_r0_anchor_layout<double>(c->at<double>(c->L.M[c->cur]), (double *)M,
                                                                c->at<int32_t>(c->L.r0cpos),
                                                                r0_cst<double>(c, 0.0, 0), 0, c->r0s.per_anchor(),
                                                                c->r0s.nthr, false, c->stream),
               "layout of Mb");
    } else if (M && n_state(c) > 0 && c->p.rc > 0) {  // tiled -> caller layout
        const int64_t nxy = (int64_t)c->p.nx * c->p.ny;
        const int vx = r0_vx(c->esz, c->r0.lmax);
        HIPCHK(c, c->esz == 4 ? launch_r0_layout<float>(c->at<float>(c->L.M[c->cur]), (float *)M, c->r0.ncell, nxy, vx, false, c->stream)
                              : launch_r0_layout<double>(c->at<double>(c->L.M[c->cur]), (double *)M, c->r0.ncell, nxy, vx, false, c->stream),
               "layout of Mb");
    } else if (M && n_state(c) > 0) {
        HIPCHK(c, hipMemcpyAsync(M, c->ws + c->L.M[c->cur], (size_t)n_state(c) * c->esz, hipMemcpyDeviceToDevice,
                                 c->stream), "copy of M");
    }
    return MMK_OK;
}

mmk_status mmk_get_stress(mmk_ctx *c, void *sigma) {
    if (!c) return MMK_ERR_ARG;
    if (!sigma) return fail(c, MMK_ERR_ARG, "sigma is NULL");
    if (!c->have_out) return fail(c, MMK_ERR_STATE, "no outputs: run mmk_step with K > 0 first");
    HIPCHK(c, hipMemcpyAsync(sigma, c->ws + c->L.stress, 3 * (size_t)c->p.nx * c->p.ny * c->esz,
                             hipMemcpyDeviceToDevice, c->stream), "copy of stress");
    return MMK_OK;
}

mmk_status mmk_get_moments(mmk_ctx *c, void *mom) {
    if (!c) return MMK_ERR_ARG;
    if (!mom) return fail(c, MMK_ERR_ARG, "moments is NULL");
    if (!c->have_out) return fail(c, MMK_ERR_STATE, "no outputs: run mmk_step with K > 0 first");
    HIPCHK(c, hipMemcpyAsync(mom, c->ws + c->L.mom, 7 * (size_t)c->p.nx * c->p.ny * c->esz,
                             hipMemcpyDeviceToDevice, c->stream), "copy of moments");
    return MMK_OK;
}

mmk_status mmk_get_motor_moments(mmk_ctx *c, void *m0, void *m1) {
    if (!c) return MMK_ERR_ARG;
    if (!c->have_out) return fail(c, MMK_ERR_STATE, "no outputs: run mmk_step with K > 0 first");
    const size_t np = (size_t)n_psi(c->p) * c->esz;
    if (m0)
        HIPCHK(c, hipMemcpyAsync(m0, c->ws + c->L.m0, np, hipMemcpyDeviceToDevice, c->stream), "copy of m0");
    if (m1) HIPCHK(c, hipMemcpyAsync(m1, c->ws + c->L.m1, np, hipMemcpyDeviceToDevice, c->stream), "copy of m1");
    return MMK_OK;
}

mmk_status mmk_get_force(mmk_ctx *c, void *force) {
    if (!c) return MMK_ERR_ARG;
    if (!force) return fail(c, MMK_ERR_ARG, "force is NULL");
    if (!c->have_state) return fail(c, MMK_ERR_STATE, "mmk_get_force before mmk_set_state");
    const mmk_params &p = c->p;
    const ForcePlan &fp = c->fplan;
    if (!c->frec_ok || fp.nt == 0)
        return fail(c, MMK_ERR_UNSUPPORTED, "spreading window of %d x %d cells is too large", fp.wx, fp.wy);
    if (p.rc > 0 && r0_field_lds(p.ns, c->esz) > 160 * 1024)
        return fail(c, MMK_ERR_UNSUPPORTED, "ns too large for the anchor-marginal field kernel at this precision");
    hipError_t e;
    // The field kernel reads the tiled layout.  After one-pass steps the state is in the anchor
    // layout: a tiled copy goes to the other M buffer (free between steps) and the state stays as
    // it is, so that the next step needs no conversion.
    size_t Mtiled = c->L.M[c->cur];
    if (p.rc > 0 && c->r0_anch) {
        const int vx = r0_vx(c->esz, c->r0.lmax), b = 1 - c->cur;
        if (c->esz == 4)
            e = launch_r0_anchor_layout<float>(c->at<float>(c->L.M[c->cur]), c->at<float>(c->L.M[b]),
                                               c->at<int32_t>(c->L.r0cpos), r0_cst<float>(c, 0.0, 0), vx,
                                               c->r0s.per_anchor(), c->r0s.nthr, false, c->stream);
        else
            e = launch_r0_anchor_layout<double>(c->at<double>(c->L.M[c->cur]), c->at<double>(c->L.M[b]),
                                                c->at<int32_t>(c->L.r0cpos), r0_cst<double>(c, 0.0, 0), vx,
                                                c->r0s.per_anchor(), c->r0s.nthr, false, c->stream);
        HIPCHK(c, e, "anchor -> tiled layout of Mb");
        Mtiled = c->L.M[b];
    }
    int slot;
    HIPCHK(c, prof_begin(c, 5, &slot), "hipEventRecord");
    // the anchor-resolved model spreads its anchor marginal (the r0 integral of Eq. (10))
    const size_t Msrc = p.rc > 0 ? c->L.Mmarg : c->L.M[c->cur];
    if (p.rc > 0) {
        if (c->esz == 4)
            e = launch_r0_field<float>(c->at<float>(Mtiled), c->at<float>(c->L.Mmarg), c->at<R0Seg>(c->L.r0seg),
                                       c->at<int32_t>(c->L.r0start), r0_cst<float>(c, 0.0, 0), p.ns, c->stream);
        else
            e = launch_r0_field<double>(c->at<double>(Mtiled), c->at<double>(c->L.Mmarg),
                                        c->at<R0Seg>(c->L.r0seg), c->at<int32_t>(c->L.r0start),
                                        r0_cst<double>(c, 0.0, 0), p.ns, c->stream);
        HIPCHK(c, e, "anchor-marginal field launch");
    }
    const uint32_t *blk = c->at<uint32_t>(c->L.fblk);
    const int *exy = c->at<int>(c->L.fexy);
    const double *cs = c->at<double>(c->L.fcs);
    if (c->esz == 4)
        e = launch_motor_force<float>(c->at<float>(Msrc), c->at<float>(c->L.psi[c->cur]), blk, exy, cs,
                                      c->at<double>(c->L.fpart), (float *)force, p.nx, p.ny, p.ntheta, p.ns, p.F,
                                      p.L, fp, c->stream);
    else
        e = launch_motor_force<double>(c->at<double>(Msrc), c->at<double>(c->L.psi[c->cur]), blk, exy, cs,
                                       c->at<double>(c->L.fpart), (double *)force, p.nx, p.ny, p.ntheta, p.ns, p.F,
                                       p.L, fp, c->stream);
    if (e == hipErrorInvalidValue)
        return fail(c, MMK_ERR_UNSUPPORTED, "spreading window of %zu bytes exceeds the LDS per block", fp.lds_bytes);
    HIPCHK(c, e, "motor force launch");
    HIPCHK(c, prof_end(c, 5, slot), "hipEventRecord");
    return MMK_OK;
}

mmk_status mmk_get_anchors(mmk_ctx *c, void *coarse, void *free_pool) {
    if (!c) return MMK_ERR_ARG;
    if (c->p.rc == 0) return fail(c, MMK_ERR_STATE, "mmk_get_anchors needs the anchor-resolved model (rc > 0)");
    if (!c->have_state) return fail(c, MMK_ERR_STATE, "mmk_get_anchors before mmk_set_state");
    if (!coarse && !free_pool) return MMK_OK;
    return c->esz == 4 ? r0_anchors<float>(c, false, (float *)coarse, (float *)free_pool)
                       : r0_anchors<double>(c, false, (double *)coarse, (double *)free_pool);
}

int64_t mmk_r0_cells(const mmk_params *p, int32_t *cells) {
    if (!check_params(p).empty() || !(p->rc > 0)) return -1;
    const R0Plan rp = r0_plan_of(*p, true);
    if (!rp.ok) return -1;
    if (cells && rp.ncell > 0) std::memcpy(cells, rp.cells.data(), rp.cells.size() * sizeof(int32_t));
    return rp.ncell;
}

mmk_status mmk_get_sums(mmk_ctx *c, double *mass, double sum_sigma[3]) {
    if (!c) return MMK_ERR_ARG;
    if (!c->have_out) return fail(c, MMK_ERR_STATE, "no outputs: run mmk_step with K > 0 first");
    if (c->sums_pending) {
        const mmk_status st = c->esz == 4 ? global_sums<float>(c) : global_sums<double>(c);
        if (st != MMK_OK) return st;
        c->sums_pending = false;
    }
    double h[4];
    HIPCHK(c, hipMemcpyAsync(h, c->ws + c->L.sums, sizeof h, hipMemcpyDeviceToHost, c->stream), "copy of sums");
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (mass) *mass = h[0];
    if (sum_sigma) {
        sum_sigma[0] = h[1];
        sum_sigma[1] = h[2];
        sum_sigma[2] = h[3];
    }
    return MMK_OK;
}

mmk_status mmk_tape_begin(mmk_ctx *c, int32_t ckpt_every) {
    if (!c) return MMK_ERR_ARG;
    if (c->p.rc > 0)
        return fail(c, MMK_ERR_UNSUPPORTED, "the adjoint covers the anchor-marginal model only (rc = 0)");
    if (c->p.m_total > 0)
        return fail(c, MMK_ERR_UNSUPPORTED, "the adjoint covers linear attachment only (m_total = 0)");
    if (c->p.motor_cfl > 0)
        return fail(c, MMK_ERR_UNSUPPORTED, "the adjoint covers one motor step per micro-step (motor_cfl = 0)");
    return tape_begin(c, &c->tape, ckpt_every, c->have_state, c->have_fluid, c->cur);
}

mmk_status mmk_tape_backward(mmk_ctx *c, const void *g_sigma, const void *g_moments, void *g_psi0,
                             double g_params[3]) {
    if (!c) return MMK_ERR_ARG;
    return c->esz == 4 ? tape_backward<float>(c, &c->tape, g_sigma, g_moments, g_psi0, g_params)
                       : tape_backward<double>(c, &c->tape, g_sigma, g_moments, g_psi0, g_params);
}

mmk_status mmk_tape_end(mmk_ctx *c) {
    if (!c) return MMK_ERR_ARG;
    c->tape.active = false;
    c->tape.steps = 0;
    return MMK_OK;
}

mmk_status mmk_profile(mmk_ctx *c, int32_t enable) {
    if (!c) return MMK_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (enable < 0) return fail(c, MMK_ERR_ARG, "enable must be >= 0");
    c->prof = enable != 0;
    for (int i = 0; i < kProfIds; ++i) c->nev[i] = 0, c->seen[i] = 0, c->prof_every[i] = enable > 0 ? enable : 1;
    return MMK_OK;
}

mmk_status mmk_profile_every(mmk_ctx *c, int32_t id, int32_t every) {
    if (!c) return MMK_ERR_ARG;
    if (id < 0 || id >= kProfIds) return fail(c, MMK_ERR_ARG, "kernel id out of range");
    if (every < 0) return fail(c, MMK_ERR_ARG, "every must be >= 0");
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    c->prof_every[id] = every;
    c->nev[id] = 0;
    c->seen[id] = 0;
    return MMK_OK;
}

mmk_status mmk_profile_read(mmk_ctx *c, int32_t id, double *total_ms, int64_t *launches) {
    if (!c) return MMK_ERR_ARG;
    if (id < 0 || id >= kProfIds) return fail(c, MMK_ERR_ARG, "kernel id out of range");
    if (!total_ms || !launches) return fail(c, MMK_ERR_ARG, "NULL output");
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    double tot = 0;
    for (int i = 0; i < c->nev[id]; ++i) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[id][2 * i], c->ev[id][2 * i + 1]), "hipEventElapsedTime");
        tot += ms;
    }
    *total_ms = tot;
    *launches = c->nev[id];
    return MMK_OK;
}

}  // extern "C"

namespace mmk {
void set_create_error(const char *msg) { g_create_error = msg; }
}  // namespace mmk

extern "C" {
const char *mmk_last_error(const mmk_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
