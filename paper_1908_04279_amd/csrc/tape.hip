// Adjoint tape bookkeeping (host side): workspace regions, checkpoint copies, fluid slots.
#include "tape.h"

#include "adjoint.h"
#include "consts.h"

#include <cstdio>

namespace mmk {

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t tape_layout(TapeLayout *t, size_t off, size_t nm, size_t np, size_t nxy, size_t e, int C, int max_steps) {
    *t = TapeLayout{};
    if (C <= 0) return off;
    t->C = C;
    t->max_steps = max_steps;
    t->nck = max_steps / C + 1;
    t->nfluid = max_steps + 1;
    t->psi_bytes = a256(np * e);
    t->M_bytes = a256(nm * e);
    t->fluid_bytes = a256(6 * nxy * e);
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = a256(off + bytes);
        return o;
    };
    t->ck_psi = take(t->psi_bytes * t->nck);
    t->ck_M = take(t->M_bytes * t->nck);
    t->seg_psi = take(t->psi_bytes * C);
    t->seg_M = take(t->M_bytes * C);
    t->seg_m0 = take(t->psi_bytes * C);
    t->lamM[0] = take(t->M_bytes);
    t->lamM[1] = take(t->M_bytes);
    t->lamPsi[0] = take(t->psi_bytes);
    t->lamPsi[1] = take(t->psi_bytes);
    t->lam_m0 = take(t->psi_bytes);
    t->lam_m1 = take(t->psi_bytes);
    t->fluid = take(t->fluid_bytes * t->nfluid);
    t->gpart_blocks = (int)motor_reverse_blocks((int64_t)np, (int)(nm / np), (int)e);
    t->gpart = take((size_t)t->gpart_blocks * 4 * sizeof(double));
    t->gsum = take(4 * sizeof(double));
    return off;
}

void tape_init(TapeState *t, int C, int max_steps) {
    *t = TapeState{};
    t->C = C;
    t->max_steps = max_steps;
}

static mmk_status save_checkpoint(mmk_ctx *c, int slot) {
    const TapeLayout &L = ctx_tape_layout(c);
    const mmk_params &p = ctx_params(c);
    const size_t e = ctx_esz(c);
    const size_t np = (size_t)p.nx * p.ny * p.ntheta * e, nm = np * p.ns;
    char *ws = ctx_ws(c);
    hipError_t r = hipMemcpyAsync(ws + L.ck_psi + slot * L.psi_bytes, ctx_cur_psi(c), np, hipMemcpyDeviceToDevice,
                                  ctx_stream(c));
    if (r == hipSuccess)
        r = hipMemcpyAsync(ws + L.ck_M + slot * L.M_bytes, ctx_cur_M(c), nm, hipMemcpyDeviceToDevice, ctx_stream(c));
    if (r != hipSuccess) return ctx_hipfail(c, r, "checkpoint copy");
    return MMK_OK;
}

static mmk_status save_fluid(mmk_ctx *c, int slot) {
    const TapeLayout &L = ctx_tape_layout(c);
    const mmk_params &p = ctx_params(c);
    const size_t nxy = (size_t)p.nx * p.ny * ctx_esz(c);
    char *dst = ctx_ws(c) + L.fluid + slot * L.fluid_bytes;
    hipError_t r = hipMemcpyAsync(dst, ctx_fluid_u(c), 2 * nxy, hipMemcpyDeviceToDevice, ctx_stream(c));
    if (r == hipSuccess)
        r = hipMemcpyAsync(dst + 2 * nxy, ctx_fluid_G(c), 4 * nxy, hipMemcpyDeviceToDevice, ctx_stream(c));
    if (r != hipSuccess) return ctx_hipfail(c, r, "fluid record copy");
    return MMK_OK;
}

mmk_status tape_begin(mmk_ctx *c, TapeState *t, int C, bool have_state, bool have_fluid, int cur) {
    (void)cur;
    if (t->C <= 0) return ctx_fail(c, MMK_ERR_STATE, "context was created without tape space (ckpt_every = 0)");
    if (C != t->C) return ctx_fail(c, MMK_ERR_ARG, "ckpt_every differs from the value given at mmk_create");
    if (!have_state || !have_fluid) return ctx_fail(c, MMK_ERR_STATE, "tape_begin needs state and fluid set");
    t->active = true;
    t->steps = 0;
    t->step_slot.clear();
    t->step_dt.clear();
    t->nfluid = 1;
    t->cur_slot = 0;
    t->steps_on_slot = 0;
    mmk_status st = save_checkpoint(c, 0);
    if (st != MMK_OK) return st;
    return save_fluid(c, 0);
}

mmk_status tape_on_fluid(mmk_ctx *c, TapeState *t) {
    if (!t->active) return MMK_OK;
    if (t->steps_on_slot > 0) {
        if (t->nfluid >= ctx_tape_layout(c).nfluid)
            return ctx_fail(c, MMK_ERR_ARG, "more fluid exchanges than the tape can hold");
        t->cur_slot = t->nfluid++;
        t->steps_on_slot = 0;
    }
    return save_fluid(c, t->cur_slot);
}

mmk_status tape_before_step(mmk_ctx *c, TapeState *t, double dt) {
    (void)c;
    if (!t->active) return MMK_OK;
    t->step_slot.push_back(t->cur_slot);
    t->step_dt.push_back(dt);
    t->steps_on_slot++;
    return MMK_OK;
}

mmk_status tape_after_step(mmk_ctx *c, TapeState *t) {
    if (!t->active) return MMK_OK;
    t->steps++;
    if (t->steps % t->C == 0) return save_checkpoint(c, t->steps / t->C);
    return MMK_OK;
}

#define TAPE_HIP(call, what)                           \
    do {                                                \
        hipError_t _e = (call);                         \
        if (_e != hipSuccess) return ctx_hipfail(c, _e, what); \
    } while (0)

// Reverse pass over the taped run, segment by segment from the last: recompute the segment's
// forward states from its checkpoint, then step backwards through it with the reverse
// kernels.  lam_psi, lam_M ping-pong; lam_m0 carries dL/dm0 of the step's new motor state.
template <typename T>
mmk_status tape_backward(mmk_ctx *c, TapeState *t, const void *g_sigma, const void *g_moments, void *g_psi0,
                         double g_params[3]) {
    if (!t->active) return ctx_fail(c, MMK_ERR_STATE, "tape_backward without tape_begin");
    if (t->steps == 0 || !ctx_have_out(c))
        return ctx_fail(c, MMK_ERR_STATE, "tape_backward needs at least one taped step");
    if (!g_psi0 || !g_params) return ctx_fail(c, MMK_ERR_ARG, "g_psi0 or g_params is NULL");
    const mmk_params &p = ctx_params(c);
    const TapeLayout &L = ctx_tape_layout(c);
    hipStream_t s = ctx_stream(c);
    char *ws = ctx_ws(c);
    const int64_t npsi = (int64_t)p.nx * p.ny * p.ntheta, nxy = (int64_t)p.nx * p.ny;
    const size_t e = sizeof(T);
    auto P = [&](size_t off) { return reinterpret_cast<T *>(ws + off); };
    const T *tab = reinterpret_cast<const T *>(ctx_tab(c));
    const double dth = kTwoPi / p.ntheta;
    const int N = t->steps, C = t->C;

    TAPE_HIP(launch_seed<T>((const T *)g_sigma, (const T *)g_moments, (const T *)ctx_cur_psi(c),
                            (const T *)ctx_m0(c), (const T *)ctx_m1(c), tab, P(L.lamPsi[0]), P(L.lam_m0),
                            P(L.lam_m1), npsi, p.ntheta, nxy, (T)p.F, (T)p.sigma_f, (T)dth, s),
             "seed launch");
    TAPE_HIP(launch_zero_f64(reinterpret_cast<double *>(ws + L.gpart), (int64_t)L.gpart_blocks * 4, s), "zero");
    int a = 0, am = 0;
    bool have_lamM = false;
    const int nseg = (N + C - 1) / C;
    const double inv_ds = p.ns / p.L;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int c0 = seg * C, len = (N - c0 < C) ? N - c0 : C;
        T *ckpsi = P(L.ck_psi + seg * L.psi_bytes), *ckM = P(L.ck_M + seg * L.M_bytes);
        auto seg_psi = [&](int j) { return P(L.seg_psi + j * L.psi_bytes); };
        auto seg_M = [&](int j) { return P(L.seg_M + j * L.M_bytes); };
        auto seg_m0 = [&](int j) { return P(L.seg_m0 + j * L.psi_bytes); };
        auto fluid_u = [&](int n) { return P(L.fluid + t->step_slot[n] * L.fluid_bytes); };
        auto fluid_G = [&](int n) { return fluid_u(n) + 2 * nxy; };
        // recompute: states n+1 = c0+1 .. c0+len into slots 0 .. len-1, m0 of each new state
        for (int j = 0; j < len; ++j) {
            const int n = c0 + j;
            const T *Min = j == 0 ? ckM : seg_M(j - 1);
            const T *pin = j == 0 ? ckpsi : seg_psi(j - 1);
            mmk_status st = ctx_forward_step<T>(c, Min, seg_M(j), pin, seg_psi(j), seg_m0(j), fluid_u(n), fluid_G(n),
                                                t->step_dt[n]);
            if (st != MMK_OK) return st;
        }
        // reverse steps n = c0+len-1 .. c0
        for (int j = len - 1; j >= 0; --j) {
            const int n = c0 + j;
            const bool last = (n == N - 1);
            const double dt = t->step_dt[n];
            const T *psi_n = j == 0 ? ckpsi : seg_psi(j - 1);
            const T *M_n = j == 0 ? ckM : seg_M(j - 1);
            int slot;
            TAPE_HIP(ctx_prof_begin(c, 3, &slot), "hipEventRecord");
            TAPE_HIP(launch_psi_reverse<T>(P(L.lamPsi[a]), psi_n, seg_m0(j), fluid_u(n), fluid_G(n), tab,
                                           P(L.lamPsi[1 - a]), P(L.lam_m0), last, psi_const<T>(p, dt),
                                           ctx_psi_launch_rev(c), s),
                     "reverse psi launch");
            TAPE_HIP(ctx_prof_end(c, 3, slot), "hipEventRecord");
            TAPE_HIP(ctx_prof_begin(c, 4, &slot), "hipEventRecord");
            TAPE_HIP(launch_motor_reverse<T>(M_n, have_lamM ? P(L.lamM[am]) : nullptr, P(L.lam_m0),
                                             last ? P(L.lam_m1) : nullptr, P(L.lamM[1 - am]),
                                             reinterpret_cast<double *>(ws + L.gpart), L.gpart_blocks, npsi, p.ns,
                                             p.limiter, motor_const<T>(p, dt), inv_ds, s),
                     "reverse motor launch");
            TAPE_HIP(ctx_prof_end(c, 4, slot), "hipEventRecord");
            a ^= 1;
            am ^= 1;
            have_lamM = true;
        }
    }
    TAPE_HIP(hipMemcpyAsync(g_psi0, P(L.lamPsi[a]), (size_t)npsi * e, hipMemcpyDeviceToDevice, s), "copy g_psi0");
    TAPE_HIP(launch_reduce_partials(reinterpret_cast<double *>(ws + L.gpart), L.gpart_blocks,
                                    reinterpret_cast<double *>(ws + L.gsum), 1.0, 1.0, s),
             "parameter gradient sum");
    double h[4];
    TAPE_HIP(hipMemcpyAsync(h, ws + L.gsum, sizeof h, hipMemcpyDeviceToHost, s), "copy g_params");
    TAPE_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    g_params[0] = h[0];
    g_params[1] = h[1];
    g_params[2] = h[2];
    return MMK_OK;
}
template mmk_status tape_backward<float>(mmk_ctx *, TapeState *, const void *, const void *, void *, double *);
template mmk_status tape_backward<double>(mmk_ctx *, TapeState *, const void *, const void *, void *, double *);

}  // namespace mmk
