// Host build of the solvers' scalar steps (solver_ctl.h) and of the host
// loop's chunk sizing (chunking.h) for the CPU tests:
// a control block (or a family of them, for the multi-shift CG) is driven
// with reduction totals chosen by the test, and its fields are read back by
// name.  Compiled by the tests with a host C++ compiler; not part of the
// library.
#include <cstddef>
#include <cstring>

#include "chunking.h"
#include "solver_ctl.h"

using lqcd::Ctl;

namespace {

struct Field {
    const char* name;
    size_t off;
    int is_int;
};

#define D(f) {#f, offsetof(Ctl, f), 0}
#define I(f) {#f, offsetof(Ctl, f), 1}
const Field kFields[] = {
    D(bb), D(thresh), D(zz), D(ww), D(rr), D(alpha), D(beta), D(rr_max), D(delta2), D(tol2), D(true_rr),
    D(tt), D(sigma), D(zeta_prev), D(zeta), D(zeta_next), D(alpha_prev), D(beta_prev), D(rr_prev_upd),
    D(rr_outer), D(tol_inner2), D(eo_rr), D(bbh),
    {"rho_re", offsetof(Ctl, rho), 0}, {"rho_im", offsetof(Ctl, rho) + 8, 0},
    {"rho_old_re", offsetof(Ctl, rho_old), 0}, {"rho_old_im", offsetof(Ctl, rho_old) + 8, 0},
    {"balpha_re", offsetof(Ctl, balpha), 0}, {"balpha_im", offsetof(Ctl, balpha) + 8, 0},
    {"omega_re", offsetof(Ctl, omega), 0}, {"omega_im", offsetof(Ctl, omega) + 8, 0},
    {"omega_step_re", offsetof(Ctl, omega_step), 0}, {"omega_step_im", offsetof(Ctl, omega_step) + 8, 0},
    {"bl_beta_re", offsetof(Ctl, bl_beta), 0}, {"bl_beta_im", offsetof(Ctl, bl_beta) + 8, 0},
    {"bl_tau_re", offsetof(Ctl, bl_tau), 0}, {"bl_tau_im", offsetof(Ctl, bl_tau) + 8, 0},
    {"bl_gp1_re", offsetof(Ctl, bl_gp1), 0}, {"bl_gp1_im", offsetof(Ctl, bl_gp1) + 8, 0},
    {"bl_gp2_re", offsetof(Ctl, bl_gp2), 0}, {"bl_gp2_im", offsetof(Ctl, bl_gp2) + 8, 0},
    {"bl_g1_re", offsetof(Ctl, bl_g1), 0}, {"bl_g1_im", offsetof(Ctl, bl_g1) + 8, 0},
    {"bl_g2_re", offsetof(Ctl, bl_g2), 0}, {"bl_g2_im", offsetof(Ctl, bl_g2) + 8, 0},
    D(bl_sigma1), I(bl_skip),
    I(ms_index), I(ms_n), I(ms_base), I(iter), I(done), I(status), I(update), I(nupdates), I(iter_limit),
    I(lucky), I(last_upd_iter), I(stag_window), I(max_stag), I(nstag), I(reset_p), I(outer_req), I(nouter),
    I(fallback_ok),
};
#undef D
#undef I

const Field* find(const char* name)
{
    for (const Field& f : kFields)
        if (std::strcmp(f.name, name) == 0) return &f;
    return nullptr;
}

}  // namespace

extern "C" {

size_t ctl_size() { return sizeof(Ctl); }

// Control blocks ctl[0..n) as a solve starts them; with n > 1 (or shifts
// given) a multi-shift family whose base is the smallest shift.
void ctl_init(void* buf, int n, double tol, double delta, double tol_inner, int iter_limit, int stag_window,
              int max_stag, int fallback_ok, const double* shifts)
{
    lqcd::CtlInit in{};
    in.tol = tol;
    in.delta = delta;
    in.tol_inner = tol_inner;
    in.iter_limit = iter_limit;
    in.stag_window = stag_window;
    in.max_stag = max_stag;
    in.fallback_ok = fallback_ok;
    Ctl* c = static_cast<Ctl*>(buf);
    int base = 0;
    for (int i = 0; i < n; ++i) {
        c[i] = lqcd::ctl_make(in);
        if (shifts && shifts[i] < shifts[base]) base = i;
    }
    for (int i = 0; i < n; ++i) {
        c[i].sigma = shifts ? shifts[i] - shifts[base] : 0.0;
        c[i].ms_index = i;
        c[i].ms_n = n;
        c[i].ms_base = base;
    }
}

void ctl_fin(void* buf, int idx, int fin, double v0, double v1, double v2)
{
    double v[6] = {v0, v1, v2, 0.0, 0.0, 0.0};
    lqcd::finalize_totals(fin, static_cast<Ctl*>(buf) + idx, v);
}

// Up to six totals (the five of BiCGStab(2)'s Gram step).
void ctl_fin_v(void* buf, int idx, int fin, const double* vals, int n)
{
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < n && j < 6; ++j) v[j] = vals[j];
    lqcd::finalize_totals(fin, static_cast<Ctl*>(buf) + idx, v);
}

// Field by name (NaN-free doubles; ints widened); returns -1e300 for an unknown name.
double ctl_get(const void* buf, int idx, const char* name)
{
    const Field* f = find(name);
    if (!f) return -1e300;
    const char* p = reinterpret_cast<const char*>(static_cast<const Ctl*>(buf) + idx) + f->off;
    if (f->is_int) {
        int v;
        std::memcpy(&v, p, sizeof v);
        return v;
    }
    double v;
    std::memcpy(&v, p, sizeof v);
    return v;
}

int ctl_set(void* buf, int idx, const char* name, double value)
{
    const Field* f = find(name);
    if (!f) return -1;
    char* p = reinterpret_cast<char*>(static_cast<Ctl*>(buf) + idx) + f->off;
    if (f->is_int) {
        const int v = (int)value;
        std::memcpy(p, &v, sizeof v);
    } else {
        std::memcpy(p, &value, sizeof value);
    }
    return 0;
}

int ctl_fin_code(const char* name)
{
    struct {
        const char* n;
        int v;
    } t[] = {{"STORE", lqcd::FIN_STORE},       {"CG_ZZ", lqcd::FIN_CG_ZZ},       {"CG_ALPHA", lqcd::FIN_CG_ALPHA},
             {"CG_RR", lqcd::FIN_CG_RR},       {"CG_BETA", lqcd::FIN_CG_BETA},   {"TRUE_RR", lqcd::FIN_TRUE_RR},
             {"BI_ALPHA", lqcd::FIN_BI_ALPHA}, {"BI_OMEGA", lqcd::FIN_BI_OMEGA}, {"BI_RHO", lqcd::FIN_BI_RHO},
             {"BI_INIT", lqcd::FIN_BI_INIT},   {"RU_RR", lqcd::FIN_RU_RR},       {"BB_E", lqcd::FIN_BB_E},
             {"BB", lqcd::FIN_BB},             {"BB_FULL", lqcd::FIN_BB_FULL},   {"RR_INIT", lqcd::FIN_RR_INIT},
             {"MS_INIT", lqcd::FIN_MS_INIT},   {"MS_INIT_KEEP", lqcd::FIN_MS_INIT_KEEP},
             {"MS_ALPHA", lqcd::FIN_MS_ALPHA}, {"MS_BETA", lqcd::FIN_MS_BETA},
             {"BL_INIT", lqcd::FIN_BL_INIT},   {"BL_ALPHA", lqcd::FIN_BL_ALPHA}, {"BL_BETA", lqcd::FIN_BL_BETA},
             {"BL_TAU", lqcd::FIN_BL_TAU},     {"BL_OMEGA", lqcd::FIN_BL_OMEGA}, {"BL_RES", lqcd::FIN_BL_RES},
             {"EO_RR", lqcd::FIN_EO_RR},       {"BBHAT", lqcd::FIN_BBHAT}};
    for (auto& e : t)
        if (std::strcmp(e.n, name) == 0) return e.v;
    return -1;
}

int ctl_status_fallback() { return lqcd::kStatusFallback; }

// The host loop's chunk sizing.
int chunk_iterations_left(double rr_prev, int it_prev, double rr, int it, double thresh)
{
    return lqcd::iterations_left(rr_prev, it_prev, rr, it, thresh);
}
int chunk_next(int need, int in_flight, int chunk) { return lqcd::next_chunk(need, in_flight, chunk); }
}
