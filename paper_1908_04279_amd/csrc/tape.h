// Adjoint tape: checkpoints of (psi, M) every C micro-steps in the caller's workspace, the
// fluid field of every exchange, and the host-side list of (fluid slot, dt) per step.
#pragma once
#include "../../include/mmk.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <vector>

namespace mmk {

struct TapeLayout {
    int C = 0, max_steps = 0, nck = 0, nfluid = 0;
    size_t ck_psi = 0, ck_M = 0;          // nck slots each
    size_t seg_psi = 0, seg_M = 0, seg_m0 = 0;  // C slots each
    size_t lamM[2] = {0, 0}, lamPsi[2] = {0, 0}, lam_m0 = 0, lam_m1 = 0;
    size_t fluid = 0;                     // nfluid slots of u [2][nx][ny] then gradu [4][nx][ny]
    size_t gpart = 0;                     // FP64 [gpart_blocks][4] parameter-gradient partials
    size_t gsum = 0;                      // FP64 [4]
    int gpart_blocks = 0;
    size_t psi_bytes = 0, M_bytes = 0, fluid_bytes = 0;
};

struct TapeState {
    int C = 0, max_steps = 0;
    bool active = false;
    int steps = 0;
    int nfluid = 0, cur_slot = 0, steps_on_slot = 0;
    std::vector<int> step_slot;
    std::vector<double> step_dt;
};

// Reserves the tape regions after `off`; returns the new end offset.
size_t tape_layout(TapeLayout *t, size_t off, size_t nm, size_t np, size_t nxy, size_t e, int C, int max_steps);
void tape_init(TapeState *t, int C, int max_steps);

// Accessors into the context (mmk_api.hip).
const mmk_params &ctx_params(const mmk_ctx *c);
hipStream_t ctx_stream(const mmk_ctx *c);
char *ctx_ws(const mmk_ctx *c);
size_t ctx_esz(const mmk_ctx *c);
const TapeLayout &ctx_tape_layout(const mmk_ctx *c);
void *ctx_cur_M(const mmk_ctx *c);
void *ctx_cur_psi(const mmk_ctx *c);
void *ctx_fluid_u(const mmk_ctx *c);
void *ctx_fluid_G(const mmk_ctx *c);
void *ctx_m0(const mmk_ctx *c);
void *ctx_m1(const mmk_ctx *c);
void *ctx_tab(const mmk_ctx *c);
const PsiLaunch &ctx_psi_launch(const mmk_ctx *c);
const PsiLaunch &ctx_psi_launch_rev(const mmk_ctx *c);
bool ctx_have_out(const mmk_ctx *c);
mmk_status ctx_fail(mmk_ctx *c, mmk_status st, const char *msg);
mmk_status ctx_hipfail(mmk_ctx *c, hipError_t e, const char *what);
hipError_t ctx_prof_begin(mmk_ctx *c, int id, int *slot);
hipError_t ctx_prof_end(mmk_ctx *c, int id, int slot);
template <typename T>
mmk_status ctx_forward_step(mmk_ctx *c, const T *M_in, T *M_out, const T *psi_in, T *psi_out, T *m0,
                            const T *u, const T *G, double dt);

mmk_status tape_begin(mmk_ctx *c, TapeState *t, int C, bool have_state, bool have_fluid, int cur);
mmk_status tape_on_fluid(mmk_ctx *c, TapeState *t);
mmk_status tape_before_step(mmk_ctx *c, TapeState *t, double dt);
mmk_status tape_after_step(mmk_ctx *c, TapeState *t);
template <typename T>
mmk_status tape_backward(mmk_ctx *c, TapeState *t, const void *g_sigma, const void *g_moments, void *g_psi0,
                         double g_params[3]);

}  // namespace mmk
