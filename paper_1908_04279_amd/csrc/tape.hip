// Adjoint tape bookkeeping (host side): workspace regions, checkpoint copies, fluid slots.
#include "tape.h"

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
    t->gpart_blocks = 2048;
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

template <typename T>
mmk_status tape_backward(mmk_ctx *c, TapeState *t, const void *g_sigma, const void *g_moments, void *g_psi0,
                         double g_params[3]) {
    (void)t;
    (void)g_sigma;
    (void)g_moments;
    (void)g_psi0;
    (void)g_params;
    return ctx_fail(c, MMK_ERR_UNSUPPORTED, "reverse pass not available in this build");
}
template mmk_status tape_backward<float>(mmk_ctx *, TapeState *, const void *, const void *, void *, double *);
template mmk_status tape_backward<double>(mmk_ctx *, TapeState *, const void *, const void *, void *, double *);

}  // namespace mmk
