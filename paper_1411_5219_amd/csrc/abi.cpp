// C ABI of the library: argument checks, workspace planning, the operator
// compositions (full M, Schur complement) and the Krylov solvers.
//
// The solvers keep every scalar on the device (see lqcd_fin.h): each
// iteration is a fixed sequence of kernel launches whose coefficients are
// read from the control block, so the host enqueues iterations in chunks
// (optionally replayed from a captured HIP graph) and only reads the status
// back once per chunk, overlapped with the next chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <unistd.h>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "chunking.h"
#include "lqcd.h"
#include "lqcd_device.h"
#include "lqcd_kernels.h"

using namespace lqcd;

namespace {

thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define LQCD_HIP(call)                                                                                     \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess) return set_error(LQCD_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#ifndef LQCD_PLANE_PAD
#define LQCD_PLANE_PAD 1
#endif

constexpr int kMaxRhs = 16;
constexpr int kMaxRefine = 4;                  // refinement passes of a multi-shift system
constexpr int kMaxSys = 16;                    // systems in one batched solve
constexpr int kPinned = kMaxRhs * kMaxSys;     // control blocks read back at once
constexpr int kMinBlock = 64;  // smallest block size any launcher uses (partials sizing)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Sites between consecutive planes of a field.  Planes of one site are read
// together, so their base addresses must not share their low address bits
// (they would compete for the same cache sets and memory channels): the
// stride in bytes is an odd multiple of 256 for 16-byte planes.
int64_t plane_stride(int64_t Vh)
{
    int64_t S = (int64_t)align_up((size_t)Vh, 16);
#if LQCD_PLANE_PAD
    if ((S / 16) % 2 == 0) S += 16;
#endif
    return S;
}

int make_geom(const lqcd_geom* gi, Geom* g)
{
    if (!gi) return set_error(LQCD_EINVAL, "geom is NULL");
    int64_t V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int L = gi->L[mu];
        if (L < 2 || (L & 1)) return set_error(LQCD_EINVAL, "extent L[%d] = %d must be even and >= 2", mu, L);
        if (!std::isfinite(gi->theta[mu])) return set_error(LQCD_EINVAL, "theta[%d] is not finite", mu);
        V *= L;
    }
    // one parity of an FP64 spinor field (192 bytes per site) must stay below
    // 4 GiB: every field is addressed through a 32-bit-sized buffer resource
    if (V / 2 > (int64_t)21 << 20) return set_error(LQCD_EUNSUPPORTED, "volume %lld too large for one device field", (long long)V);
    for (int mu = 0; mu < 4; ++mu) g->L[mu] = gi->L[mu];
    g->Lxh = gi->L[0] / 2;
    g->Vh = (int)(V / 2);
    g->S = plane_stride(g->Vh);
    for (int mu = 0; mu < 4; ++mu) {
        g->ph[mu][0] = std::cos(gi->theta[mu]);
        g->ph[mu][1] = std::sin(gi->theta[mu]);
    }
    return LQCD_OK;
}

int check_prec(int prec, int recon)
{
    if (prec != 64 && prec != 32 && prec != 16) return set_error(LQCD_EINVAL, "prec %d not in {64, 32, 16}", prec);
    if (recon != 18 && recon != 12) return set_error(LQCD_EINVAL, "recon %d not in {18, 12}", recon);
    if (prec == 16 && recon != 12) return set_error(LQCD_EUNSUPPORTED, "FP16 links need recon 12");
    return LQCD_OK;
}

int check_op(const lqcd_op* op)
{
    if (!op) return set_error(LQCD_EINVAL, "op is NULL");
    if (!std::isfinite(op->kappa) || !std::isfinite(op->mu)) return set_error(LQCD_EINVAL, "kappa / mu not finite");
    return check_prec(op->prec, op->recon);
}

int64_t parity_bytes(const Geom& g, int prec) { return spinor_parity_bytes(prec, g.S); }
int64_t gauge_bytes(const Geom& g, int prec, int recon) { return 8 * g.S * link_bytes(prec, recon); }

// Spin-block coefficients of the twisted-mass site term.
//   A = 1 + 2 i kappa mu gamma_5 : (1 + 2 i k m) on spins 0,1 and (1 - 2 i k m) on 2,3
//   A^+ conjugates; A^-1 = (1 - 2 i kappa mu gamma_5) / (1 + 4 kappa^2 mu^2).
SpinCoef coef_A(double k, double m, bool dag, double scale = 1.0)
{
    const double t = (dag ? -2.0 : 2.0) * k * m;
    return {{scale, scale * t}, {scale, -scale * t}};
}
SpinCoef coef_Ainv(double k, double m, bool dag, double scale = 1.0)
{
    const double n = 1.0 + 4.0 * k * k * m * m;
    const double t = (dag ? 2.0 : -2.0) * k * m;
    return {{scale / n, scale * t / n}, {scale / n, -scale * t / n}};
}
SpinCoef coef_real(double v) { return {{v, 0.0}, {v, 0.0}}; }

// Process-wide launch table: [kernel family][precision 64 / 32 / 16].
std::mutex g_launch_mu;
// Defaults measured on MI355X at 24^3x8 .. 64^3x16: whole x-rows per block
// in t-fastest order with the XCD remap for the Dslash; plain 256-wide
// blocks for the site-local kernels.
// Several right-hand sides: FP64 and FP32 single right-hand sides per
// work-item in groups of 4, FP16 tiles of 2 in groups of 4.
// The staggered hop (colour vectors of 48 / 24 / 16 bytes) gains less from
// neighbour reuse: memory order in FP64, row tiles of 192 in FP32 and FP16.
Launch g_launch[4][3] = {{{256, 1, 1, 1, 4}, {256, 1, 1, 1, 4}, {256, 1, 1, 2, 4}},
                         {{256, 0, 0, 1, 0}, {256, 0, 0, 1, 0}, {256, 0, 0, 1, 0}},
                         {{256, 1, 0, 1, 0}, {192, 1, 1, 1, 0}, {192, 1, 1, 1, 0}},
                         // several right-hand sides (the autotuner for them also tries
                         // 128- and 192-thread requests; no default beat these across
                         // 24^3x8, 32^3x8 and 48^3x12 by more than the run-to-run spread)
                         {{256, 1, 1, 1, 4}, {256, 1, 1, 1, 4}, {256, 1, 1, 2, 4}}};

int prec_slot(int prec) { return prec == 64 ? 0 : prec == 32 ? 1 : prec == 16 ? 2 : -1; }

Launch launch_for(int kernel, int prec)
{
    std::lock_guard<std::mutex> lk(g_launch_mu);
    const int k = prec_slot(prec);
    return k < 0 ? Launch{} : g_launch[kernel][k];
}

// Autotune cache: launch shapes the autotuners found, keyed by the device
// architecture, kernel family, storage precision, link reconstruction,
// lattice extents and right-hand sides (the analogue of a compiled-kernel
// cache that a later run reuses).  A launch for a key in the cache uses the
// cached shape, any other the process-wide table.  With LQCD_TUNE_CACHE set
// to a path the cache is read from that file on first use and written back
// after every autotuner run.
struct TuneKey {
    std::string arch;
    int kernel, prec, recon, L[4], nrhs;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(arch, kernel, prec, recon, L[0], L[1], L[2], L[3], nrhs) <
               std::tie(o.arch, o.kernel, o.prec, o.recon, o.L[0], o.L[1], o.L[2], o.L[3], o.nrhs);
    }
};
struct TuneVal {
    Launch l;
    double us;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
bool g_tune_env_read = false;

// Architecture of the current device without its feature suffix (gcnArchName
// "gfx950:sramecc+:xnack-" -> "gfx950"; "host" without a device), looked up
// once per device: the lookup sits on the launch path.  Callers hold g_tune_mu.
std::string device_arch()
{
    static std::map<int, std::string> known;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return "host";
    }
    const auto it = known.find(dev);
    if (it != known.end()) return it->second;
    hipDeviceProp_t prop;
    std::string a = "host";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        a = prop.gcnArchName;
        const size_t c = a.find(':');
        if (c != std::string::npos) a = a.substr(0, c);
    } else {
        (void)hipGetLastError();
    }
    known[dev] = a;
    return a;
}

TuneKey tune_key(int kernel, int prec, int recon, const int L[4], int nrhs)
{
    TuneKey k{device_arch(), kernel, prec, recon, {L[0], L[1], L[2], L[3]}, nrhs};
    return k;
}

const char* tune_env_path()
{
    const char* p = std::getenv("LQCD_TUNE_CACHE");
    return p && *p ? p : nullptr;
}

// Shape checks shared by lqcd_set_launch and the cache (returns an error message or null).
const char* launch_problem(int kernel, const Launch& c)
{
    if (c.block < 64 || c.block > 256 || c.block % 64) return "block not in {64, 128, 192, 256}";
    if (c.swizzle != 0 && c.swizzle != 1) return "swizzle must be 0 or 1";
    if (c.order < 0 || c.order > 64) return "order must be in 0..64";
    if (c.order >= 1 && kernel == LQCD_KERNEL_BLAS) return "order >= 1 applies to the hop kernels only";
    if (c.rhs_tile != 1 && c.rhs_tile != 2 && c.rhs_tile != 4) return "rhs_tile not in {1, 2, 4}";
    if (c.rhs_group != 0 && (c.rhs_group < 2 || c.rhs_group > 16)) return "rhs_group not 0 or in [2, 16]";
    if (c.ygroup < 1 || c.ygroup > 64) return "ygroup not in [1, 64]";
    if (c.rhs_lanes != 1 && c.rhs_lanes != 2 && c.rhs_lanes != 4 && c.rhs_lanes != 8 && c.rhs_lanes != 16)
        return "rhs_lanes not in {1, 2, 4, 8, 16}";
    return nullptr;
}

int tune_load_locked(const char* path, bool missing_ok)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return missing_ok ? LQCD_OK : set_error(LQCD_EINVAL, "cannot read the tune cache %s", path);
    std::map<TuneKey, TuneVal> got;
    char line[1024];
    int lineno = 0, rc = LQCD_OK;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        const char* b = std::strchr(line, '{');
        if (!b) {
            // only the brackets of the array and blank lines carry no entry
            for (const char* c = line; *c; ++c)
                if (*c != '[' && *c != ']' && *c != ' ' && *c != '\n' && *c != '\r' && *c != '\t') {
                    rc = set_error(LQCD_EINVAL, "tune cache %s line %d: not an entry", path, lineno);
                    break;
                }
            if (rc) break;
            continue;
        }
        char arch[64] = "";
        TuneKey k{};
        TuneVal v{};
        const int n = std::sscanf(
            b,
            "{\"arch\": \"%63[^\"]\", \"kernel\": %d, \"prec\": %d, \"recon\": %d, \"L\": [%d, %d, %d, %d], "
            "\"nrhs\": %d, \"block\": %d, \"swizzle\": %d, \"order\": %d, \"rhs_tile\": %d, \"rhs_group\": %d, "
            "\"ygroup\": %d, \"rhs_lanes\": %d, \"us\": %lf}",
            arch, &k.kernel, &k.prec, &k.recon, &k.L[0], &k.L[1], &k.L[2], &k.L[3], &k.nrhs, &v.l.block,
            &v.l.swizzle, &v.l.order, &v.l.rhs_tile, &v.l.rhs_group, &v.l.ygroup, &v.l.rhs_lanes, &v.us);
        const char* bad = n == 17 ? launch_problem(k.kernel, v.l) : "malformed entry";
        if (!bad && (k.kernel < 0 || k.kernel > LQCD_KERNEL_DSLASH_RHS)) bad = "unknown kernel";
        if (!bad && prec_slot(k.prec) < 0) bad = "prec not in {64, 32, 16}";
        if (!bad && k.recon != 18 && k.recon != 12) bad = "recon not 18 or 12";
        if (!bad && (k.nrhs < 1 || k.nrhs > kMaxRhs)) bad = "nrhs out of range";
        if (bad) {
            rc = set_error(LQCD_EINVAL, "tune cache %s line %d: %s", path, lineno, bad);
            break;
        }
        k.arch = arch;
        got[k] = v;
    }
    std::fclose(f);
    if (rc) return rc;
    for (const auto& e : got) g_tune[e.first] = e.second;
    return LQCD_OK;
}

int tune_save_locked(const char* path)
{
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return set_error(LQCD_EINVAL, "cannot write the tune cache %s", path);
    std::fprintf(f, "[\n");
    size_t i = 0;
    for (const auto& e : g_tune) {
        const TuneKey& k = e.first;
        const TuneVal& v = e.second;
        std::fprintf(f,
                     "{\"arch\": \"%s\", \"kernel\": %d, \"prec\": %d, \"recon\": %d, \"L\": [%d, %d, %d, %d], "
                     "\"nrhs\": %d, \"block\": %d, \"swizzle\": %d, \"order\": %d, \"rhs_tile\": %d, "
                     "\"rhs_group\": %d, \"ygroup\": %d, \"rhs_lanes\": %d, \"us\": %.3f}%s\n",
                     k.arch.c_str(), k.kernel, k.prec, k.recon, k.L[0], k.L[1], k.L[2], k.L[3], k.nrhs, v.l.block,
                     v.l.swizzle, v.l.order, v.l.rhs_tile, v.l.rhs_group, v.l.ygroup, v.l.rhs_lanes, v.us,
                     ++i < g_tune.size() ? "," : "");
    }
    std::fprintf(f, "]\n");
    const bool ok = std::fflush(f) == 0;
    std::fclose(f);
    if (!ok || std::rename(tmp.c_str(), path) != 0) return set_error(LQCD_EINVAL, "cannot write the tune cache %s", path);
    return LQCD_OK;
}

// First use: read the file LQCD_TUNE_CACHE names (a missing file is an empty cache).
void tune_env_init_locked()
{
    if (g_tune_env_read) return;
    g_tune_env_read = true;
    if (const char* p = tune_env_path()) (void)tune_load_locked(p, true);
}

// Shape for a launch of kernel family `kernel` on this problem.
Launch launch_for(int kernel, int prec, int recon, const Geom& g, int nrhs)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_env_init_locked();
        if (!g_tune.empty()) {
            const auto it = g_tune.find(tune_key(kernel, prec, recon, g.L, nrhs));
            if (it != g_tune.end()) return it->second.l;
        }
    }
    return launch_for(kernel, prec);
}

// An autotuner's result: into the cache (and its file, if LQCD_TUNE_CACHE is set).
void tune_record(int kernel, int prec, int recon, const int L[4], int nrhs, const Launch& l, double us)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_init_locked();
    g_tune[tune_key(kernel, prec, recon, L, nrhs)] = TuneVal{l, us};
    if (const char* p = tune_env_path()) (void)tune_save_locked(p);
}

// Bump allocator over the caller's workspace.
struct Arena {
    char* base;
    size_t off = 0;
    size_t cap;
    void* take(size_t bytes)
    {
        off = align_up(off, 256);
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

// Reduction scratch shared by every kernel of one call (kernels run in
// stream order, so one set of partials is enough).
struct RedScratch {
    double* partials = nullptr;
    int capacity = 0;  // blocks per right-hand side
    Ctl* ctl = nullptr;
};

// Most blocks any reducing launch uses: memory order with the smallest
// block over both parities, or row tiles of one x-row each over both
// parities (one block per (y, z, t)).
int64_t max_blocks(const Geom& g)
{
    const int64_t linear = 2 * ((g.Vh + kMinBlock - 1) / kMinBlock);
    const int64_t tiled = 2 * (int64_t)g.L[1] * g.L[2] * g.L[3];
    return linear > tiled ? linear : tiled;
}

void plan_reductions(Arena& ar, const Geom& g, int nrhs, RedScratch* rs)
{
    const int64_t nblk = max_blocks(g);
    rs->capacity = (int)nblk;
    rs->partials = static_cast<double*>(ar.take(sizeof(double) * kMaxFin * nblk * nrhs));
    rs->ctl = static_cast<Ctl*>(ar.take(sizeof(Ctl) * kMaxRhs));
}

// One operator bound to a gauge field, a precision and a stream.
struct Op {
    Geom g;
    int prec = 64, recon = 18;
    const void* U = nullptr;
    double kappa = 0, mu = 0;
    int nrhs = 1;
    int64_t pb = 0;  // bytes of one parity field at prec
    hipStream_t s = nullptr;
    RedScratch rs;
    Launch dcfg, bcfg;

    void tune()
    {
        dcfg = launch_for(nrhs > 1 ? LQCD_KERNEL_DSLASH_RHS : LQCD_KERNEL_DSLASH, prec, recon, g, nrhs);
        bcfg = launch_for(LQCD_KERNEL_BLAS, prec);
    }

    DslashArgs base() const
    {
        DslashArgs a{};
        a.g = g;
        a.U = U;
        a.st_in = a.st_out = a.st_site = a.st_add = a.st_aux = pb;
        a.par_bytes = pb;
        a.r.partials = rs.partials;
        a.r.capacity = rs.capacity;
        a.ctl = rs.ctl;
        return a;
    }

    // out(parity p) = add + a * site + c * H_{p,1-p} in     (dag: H^+)
    hipError_t hop(int p, const void* in, void* out, bool dag, SpinCoef ca, const void* site, SpinCoef cc,
                   const void* add, int red, int fin, int pred, const void* aux = nullptr) const
    {
        DslashArgs a = base();
        a.parity = p;
        a.pred = pred;
        a.in = in;
        a.out = out;
        a.site = site;
        a.add = add;
        a.aux = aux;
        a.a = ca;
        a.c = cc;
        a.r.fin = fin;
        return launch_dslash(prec, recon, dag, red, a, nrhs, dcfg, s);
    }

    // out = add + sgn * M in on full-lattice fields (M^+ for dag), one launch.
    hipError_t full_M(const void* in, void* out, bool dag, double sgn, const void* add, int red, int fin, int pred,
                      const void* aux = nullptr, int64_t st_in = -1, int64_t st_out = -1, int64_t st_add = -1,
                      int fin_even = 0) const
    {
        DslashArgs a = base();
        a.full = 1;
        a.r.fin_even = fin_even;
        a.pred = pred;
        a.in = in;
        a.site = in;
        a.out = out;
        a.add = add;
        a.aux = aux;
        a.st_in = a.st_site = st_in >= 0 ? st_in : 2 * pb;
        a.st_out = st_out >= 0 ? st_out : 2 * pb;
        a.st_add = st_add >= 0 ? st_add : 2 * pb;
        a.st_aux = 2 * pb;
        a.a = coef_A(kappa, mu, dag, sgn);
        a.c = coef_real(-sgn * kappa);
        a.r.fin = fin;
        return launch_dslash(prec, recon, dag, red, a, nrhs, dcfg, s);
    }

    // out = add + sgn * Mhat in on even parity fields, tmp an odd field.
    //   Mhat = A - kappa^2 H_eo A^-1 H_oe ;  Mhat^+ = A^+ - kappa^2 H^+_eo (A^-1)^+ H^+_oe
    hipError_t schur(const void* in, void* out, void* tmp, bool dag, double sgn, const void* add, int red, int fin,
                     int pred, const void* aux = nullptr, int64_t st_in = -1, int64_t st_add = -1) const
    {
        DslashArgs a = base();
        a.parity = 1;
        a.pred = pred;
        a.in = in;
        a.out = tmp;
        a.st_in = st_in >= 0 ? st_in : pb;
        a.c = coef_Ainv(kappa, mu, dag);
        a.r.fin = FIN_STORE;
        hipError_t e = launch_dslash(prec, recon, dag, RED_NONE, a, nrhs, dcfg, s);
        if (e != hipSuccess) return e;
        DslashArgs b = base();
        b.parity = 0;
        b.pred = pred;
        b.in = tmp;
        b.out = out;
        b.site = in;
        b.st_site = st_in >= 0 ? st_in : pb;
        b.add = add;
        b.st_add = st_add >= 0 ? st_add : pb;
        b.aux = aux;
        b.a = coef_A(kappa, mu, dag, sgn);
        b.c = coef_real(-sgn * kappa * kappa);
        b.r.fin = fin;
        return launch_dslash(prec, recon, dag, red, b, nrhs, dcfg, s);
    }

    BlasArgs blas_base(int nsub) const
    {
        BlasArgs a{};
        a.Vh = g.Vh;
        a.S = g.S;
        a.nsub = nsub;
        a.sub_stride = pb;
        const int64_t st = nsub * pb;
        a.st_x = a.st_y = a.st_z = a.st_w = a.st_v = a.st_r0 = st;
        a.r.partials = rs.partials;
        a.r.capacity = rs.capacity;
        a.ctl = rs.ctl;
        return a;
    }

    hipError_t blas(int op, int nsub, int pred, int fin, void* x, void* y = nullptr, void* z = nullptr,
                    void* w = nullptr, void* v = nullptr, const void* r0 = nullptr, SpinCoef coef = {}) const
    {
        BlasArgs a = blas_base(nsub);
        a.pred = pred;
        a.x = x;
        a.y = y;
        a.z = z;
        a.w = w;
        a.v = v;
        a.r0 = r0;
        a.coef = coef;
        a.r.fin = fin;
        return launch_blas(prec, op, a, nrhs, bcfg, s);
    }
};

#define LQCD_K(call)                                                                                         \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess) return set_error(LQCD_EHIP, "kernel launch failed (%s): %s", #call,           \
                                               hipGetErrorString(e_));                                       \
    } while (0)

// Pinned host mirror of the control blocks (per thread, allocated once).
struct Pinned {
    Ctl* buf = nullptr;  // 2 * kPinned
    ~Pinned()
    {
        if (buf) (void)hipHostFree(buf);
    }
};
thread_local Pinned g_pinned;

int pinned_ctl(Ctl** out)
{
    if (!g_pinned.buf) LQCD_HIP(hipHostMalloc((void**)&g_pinned.buf, sizeof(Ctl) * 2 * kPinned, hipHostMallocDefault));
    *out = g_pinned.buf;
    return LQCD_OK;
}

enum Method { M_CG = 0, M_BICG = 1 };

// Defaults of the stagnation handling of mixed-precision solves.
constexpr int kDefaultStagWindow = 500;   // iterations without a reliable update
constexpr int kDefaultMaxStag = 3;        // stagnations before FP16 storage falls back to FP32

int stag_window_of(const lqcd_solve_params* p)
{
    return p->stag_window == 0 ? kDefaultStagWindow : p->stag_window < 0 ? 0 : p->stag_window;
}
int max_stag_of(const lqcd_solve_params* p)
{
    return p->max_stagnations == 0 ? kDefaultMaxStag : p->max_stagnations < 0 ? 0 : p->max_stagnations;
}
// An FP16 inner solve of a single system may continue at FP32 storage.
bool may_fall_back(const lqcd_solve_params* p) { return p->inner_prec == 16 && max_stag_of(p) > 0; }

// Workspace plan of one solver call: the reductions first, then the vectors.
struct SolverPlan {
    RedScratch rs;
    void* v[12] = {};        // FP64 (or outer-precision) vectors
    void* lo[8] = {};        // low-precision vectors (mixed)
    void* Ulo = nullptr;     // low-precision gauge field (mixed)
    size_t bytes = 0;
};

int plan_solver(const Geom& g, const lqcd_op* op, const lqcd_solve_params* prm, int method, void* ws, SolverPlan* sp,
                bool single = true)
{
    Arena ar{static_cast<char*>(ws), 0, 0};
    const int nrhs = prm->nrhs;
    plan_reductions(ar, g, nrhs, &sp->rs);
    const int64_t pb = parity_bytes(g, 64);
    const bool eo = prm->eo != 0;
    const int64_t vec = (eo ? 1 : 2) * pb * nrhs;
    const bool mixed = prm->inner_prec != 64;
    // FP64 vectors: CG eo: r p w z t bhat | BiCG eo: r r0 p v s t tmp bhat
    //               CG full: r p w z     | BiCG full: r r0 p v s t
    //               BiCGStab(2) eo: r_0 r_1 r_2 u_0 u_1 u_2 rt tmp bhat (full: the first 7)
    int nv = 0;
    if (method == M_CG) nv = mixed ? 3 : (eo ? 6 : 4);
    else if (prm->bicgstab_ell == 2) nv = eo ? 9 : 7;
    else nv = eo ? 8 : 6;
    for (int i = 0; i < nv; ++i) sp->v[i] = ar.take((size_t)vec);
    if (mixed) {
        // an FP16 inner solve that may fall back to FP32 storage holds
        // FP32-sized inner fields and links from the start
        const int lp = single && may_fall_back(prm) ? 32 : prm->inner_prec;
        const int64_t lpb = parity_bytes(g, lp);
        // xl rl pl wl zl tl
        for (int i = 0; i < 6; ++i) sp->lo[i] = ar.take((size_t)(lpb * nrhs));
        sp->Ulo = ar.take((size_t)gauge_bytes(g, lp, prm->inner_recon));
    }
    (void)op;
    sp->bytes = align_up(ar.off, 256);
    return LQCD_OK;
}

int check_params(const lqcd_solve_params* p, int method)
{
    if (!p) return set_error(LQCD_EINVAL, "params is NULL");
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return set_error(LQCD_EINVAL, "tol must be > 0");
    if (p->maxiter < 0) return set_error(LQCD_EINVAL, "maxiter < 0");
    if (p->nrhs < 1 || p->nrhs > kMaxRhs) return set_error(LQCD_EINVAL, "nrhs %d not in [1, %d]", p->nrhs, kMaxRhs);
    if (p->inner_prec != 64) {
        if (method != M_CG) return set_error(LQCD_EUNSUPPORTED, "mixed precision is implemented for CG only");
        if (!p->eo) return set_error(LQCD_EUNSUPPORTED, "mixed precision needs eo = 1");
        int rc = check_prec(p->inner_prec, p->inner_recon);
        if (rc) return rc;
        if (!(p->delta_reliable > 0.0 && p->delta_reliable < 1.0))
            return set_error(LQCD_EINVAL, "delta_reliable must be in (0, 1)");
        if (!(p->tol_inner >= 0.0 && p->tol_inner < 1.0))
            return set_error(LQCD_EINVAL, "tol_inner must be in [0, 1)");
    }
    if (p->persistent < 0 || p->persistent > 2) return set_error(LQCD_EINVAL, "persistent %d not in {0, 1, 2}", p->persistent);
    if (p->bicgstab_ell < 0 || p->bicgstab_ell > 2)
        return set_error(LQCD_EINVAL, "bicgstab_ell %d not in {0, 1, 2}", p->bicgstab_ell);
    return LQCD_OK;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Runs enqueue_iter() in chunks of at most `chunk` iterations until every
// solve is done: the control blocks ctl[s * stride + r] (s < nsys, r < nrhs)
// are read back after each chunk, and the read-back of a chunk is waited
// for while the next one runs.  Near the end the chunks shrink: from two
// read-backs of each open solve the rate at which ||r||^2 falls per
// iteration gives the iterations it still needs, and the next chunk covers
// what the chunk in flight does not (at least one iteration), so few no-op
// iterations follow convergence.  With use_graph the chunk is captured once
// as a HIP graph and replayed at full length; instead of shrinking, the
// host then reads the status of the chunk in flight before replaying
// another when that chunk should finish every solve.
template <class F>
int drive(hipStream_t st, const Ctl* ctl, int nsys, int stride, int nrhs, int chunk, int maxiter, bool use_graph,
          F&& enqueue_iter)
{
    Ctl* pin = nullptr;
    int rc = pinned_ctl(&pin);
    if (rc) return rc;
    const int count = nsys * stride;
    hipEvent_t ev[2];
    LQCD_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    LQCD_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int result = LQCD_OK;
    auto enqueue_chunk = [&](int len) -> int {
        if (use_graph) {
            if (!exec) {
                LQCD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                int r = LQCD_OK;
                for (int k = 0; k < chunk && r == LQCD_OK; ++k) r = enqueue_iter();
                hipGraph_t gph = nullptr;
                hipError_t e = hipStreamEndCapture(st, &gph);
                if (r) return r;
                if (e != hipSuccess) return set_error(LQCD_EHIP, "graph capture failed: %s", hipGetErrorString(e));
                graph = gph;
                LQCD_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            }
            LQCD_HIP(hipGraphLaunch(exec, st));
            return LQCD_OK;
        }
        for (int k = 0; k < len; ++k) {
            int r = enqueue_iter();
            if (r) return r;
        }
        return LQCD_OK;
    };
    // The solver's own iteration limit ends the work (the kernels of a
    // finished solve are no-ops); this bounds the host loop.
    const int64_t max_enqueue = (int64_t)maxiter + 2 * (int64_t)chunk;
    int64_t enqueued = 0;
    int issued = 0, seen = 0;                   // chunks enqueued, chunks whose status was read
    int len[2] = {0, 0};                        // iterations of chunk i, at len[i & 1] (two in flight at most)
    std::vector<double> prev_rr(count, -1.0);  // ||r||^2 and iteration at the previous read-back
    std::vector<int> prev_it(count, -1);
    int need = -1;                              // iterations the slowest open solve still needs (-1: unknown)
    // The chunks in flight cover `out` iterations; once they cover what the
    // slowest solve needs (plus one without graph replay, whose chunks are
    // sized to it) no further chunk is queued before their status is read.
    const int margin = use_graph ? 0 : 1;
    for (;;) {
        while (enqueued < max_enqueue && issued - seen < 2) {
            int out = 0;
            for (int i = seen; i < issued; ++i) out += len[i & 1];
            if (issued > seen && need >= 0 && need + margin <= out) break;
            const int c = use_graph ? chunk : next_chunk(need, out, chunk);
            result = enqueue_chunk(c);
            if (result) break;
            const int slot = issued & 1;
            hipError_t e = hipMemcpyAsync(pin + slot * kPinned, ctl, sizeof(Ctl) * count, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipEventRecord(ev[slot], st);
            if (e != hipSuccess) { result = set_error(LQCD_EHIP, "status read-back: %s", hipGetErrorString(e)); break; }
            enqueued += c;
            len[slot] = c;
            ++issued;
        }
        if (result) break;
        if (issued == seen) break;  // the iteration bound is reached and every chunk was read
        const int m = seen & 1;
        hipError_t e = hipEventSynchronize(ev[m]);
        if (e != hipSuccess) { result = set_error(LQCD_EHIP, "stream: %s", hipGetErrorString(e)); break; }
        ++seen;
        bool all = true, known = true;
        int most = 0;
        for (int sy = 0; sy < nsys; ++sy)
            for (int i = 0; i < nrhs; ++i) {
                const int k = sy * stride + i;
                const Ctl& c = pin[m * kPinned + k];
                if (c.done) continue;
                all = false;
                const int left = iterations_left(prev_rr[k], prev_it[k], c.rr, c.iter, c.thresh);
                if (left < 0) known = false;
                else most = std::max(most, left);
                prev_rr[k] = c.rr;
                prev_it[k] = c.iter;
            }
        need = known ? most : -1;
        if (all) break;
    }
    (void)hipStreamSynchronize(st);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return result;
}

int read_ctls(hipStream_t st, const Ctl* ctl, int count, std::vector<Ctl>& out)
{
    out.resize(count);
    LQCD_HIP(hipMemcpyAsync(out.data(), ctl, sizeof(Ctl) * count, hipMemcpyDeviceToHost, st));
    LQCD_HIP(hipStreamSynchronize(st));
    return LQCD_OK;
}

// Bookkeeping shared by the solvers: which right-hand sides to reopen after
// the true-residual check, and the per-right-hand-side info.
unsigned reopen_mask(const Ctl* ctl, int nrhs, const lqcd_solve_params* prm)
{
    unsigned mask = 0;
    for (int i = 0; i < nrhs; ++i) {
        const double tr = ctl[i].bb > 0 ? std::sqrt(ctl[i].true_rr / ctl[i].bb) : 0.0;
        if (ctl[i].status == 0 && tr > prm->tol && ctl[i].iter < prm->maxiter) mask |= 1u << i;
    }
    return mask;
}

void fill_info(const Ctl* ctl, int nrhs, int method, bool eo, bool mixed, int restarts, double secs,
               const lqcd_solve_params* prm, lqcd_solve_info* info, int* worst, unsigned fallbacks = 0)
{
    for (int i = 0; i < nrhs; ++i) {
        lqcd_solve_info& in = info[i];
        in.iters = ctl[i].iter;
        in.reliable_updates = ctl[i].nupdates;
        in.restarts = restarts;
        in.true_resid = ctl[i].bb > 0 ? std::sqrt(ctl[i].true_rr / ctl[i].bb) : 0.0;
        in.eo_resid = !eo ? std::nan("") : ctl[i].bbh > 0 ? std::sqrt(ctl[i].eo_rr / ctl[i].bbh) : 0.0;
        in.seconds = secs;
        // Dslash applications (eo-hop units): eo solves apply Mhat as 2 hops,
        // full-lattice solves apply M as one launch over V = 2 x V/2 sites.
        const double it = ctl[i].iter, starts = restarts + 1;
        const double prep = eo ? 1.0 : 0.0;                 // bhat
        const double finish = (eo ? 1.0 : 0.0) + 2.0;       // reconstruct, true residual (full M)
        if (!mixed) {
            const double per_start = method == M_CG ? 4.0 : 2.0;  // residual (+ z = Op^+ r for CG)
            in.hops_outer = prep + starts * (per_start + finish) + 4.0 * it;
            in.hops_inner = 0.0;
        } else {
            in.hops_outer = prep + starts * (2.0 + finish) + 2.0 * ctl[i].nupdates;
            in.hops_inner = starts * 2.0 + 4.0 * it;
        }
        in.outer_iters = 1 + ctl[i].nouter;
        in.stagnations = ctl[i].nstag;
        in.fallbacks = fallbacks ? ((fallbacks >> i) & 1u) : 0;
        in.persistent_launches = 0;
        int st = ctl[i].status;
        if (st == LQCD_OK && in.true_resid > prm->tol) st = LQCD_ENOCONV;
        if (st == LQCD_OK && !std::isfinite(in.true_resid)) st = LQCD_ENONFINITE;
        in.status = st;
        if (st != LQCD_OK && *worst == LQCD_OK) *worst = st;
    }
}

// Set-up shared by the solvers: control blocks, ||b||^2, and (even-odd) the
// prepared source bhat = b_e + kappa H_eo A^-1 b_o with x_e = 0 (t is an odd
// scratch field); full lattice: x = 0.
int solver_setup(const Op& o, const lqcd_solve_params* prm, bool eo, bool mixed, char* bc, char* xc, void* bhat,
                 void* t, bool allow_fallback = false)
{
    const int nrhs = o.nrhs;
    const int64_t pb = o.pb, fb = 2 * pb;
    hipStream_t s = o.s;
    CtlInit ci{};
    ci.tol = prm->tol;
    ci.iter_limit = prm->maxiter;
    if (mixed) {
        ci.delta = prm->delta_reliable;
        ci.tol_inner = prm->tol_inner;
        ci.stag_window = stag_window_of(prm);
        ci.max_stag = max_stag_of(prm);
        ci.fallback_ok = allow_fallback && may_fall_back(prm) ? 1 : 0;
    }
    LQCD_K(launch_ctl_init(o.rs.ctl, nrhs, ci, s));
    {
        BlasArgs a = o.blas_base(2);
        a.pred = PRED_ALWAYS;
        a.x = bc;
        a.r.fin = FIN_BB_FULL;
        LQCD_K(launch_blas(64, BLAS_NORM, a, nrhs, o.bcfg, s));
    }
    if (eo) {
        BlasArgs a = o.blas_base(1);
        a.pred = PRED_ALWAYS;
        a.x = bc + pb;
        a.y = t;
        a.st_x = fb;
        a.coef = coef_Ainv(o.kappa, o.mu, false);
        LQCD_K(launch_blas(64, BLAS_SPIN_SCALE, a, nrhs, o.bcfg, s));
        DslashArgs d = o.base();
        d.parity = 0;
        d.pred = PRED_ALWAYS;
        d.in = t;
        d.out = bhat;
        d.add = bc;
        d.st_add = fb;
        d.c = coef_real(o.kappa);
        d.r.fin = FIN_BBHAT;  // ||bhat||^2, the scale of the even-odd residual
        LQCD_K(launch_dslash(64, o.recon, false, RED_NORM, d, nrhs, o.dcfg, s));
        BlasArgs z = o.blas_base(1);
        z.pred = PRED_ALWAYS;
        z.y = xc;
        z.st_y = fb;
        LQCD_K(launch_blas(64, BLAS_ZERO, z, nrhs, o.bcfg, s));
    } else {
        LQCD_K(o.blas(BLAS_ZERO, 2, PRED_ALWAYS, FIN_STORE, nullptr, xc));
    }
    return LQCD_OK;
}

// Solution, reconstruction and true residual: x_o = A^-1 (b_o + kappa H_oe x_e)
// (even-odd), then ||b - M x||^2 in FP64 on the full lattice.
int solver_finish(const Op& o, bool eo, char* bc, char* xc)
{
    const int64_t pb = o.pb, fb = 2 * pb;
    if (eo) {
        DslashArgs d = o.base();
        d.parity = 1;
        d.pred = PRED_ALWAYS;
        d.in = xc;
        d.st_in = fb;
        d.out = xc + pb;
        d.st_out = fb;
        d.site = bc + pb;
        d.st_site = fb;
        d.a = coef_Ainv(o.kappa, o.mu, false);
        d.c = coef_Ainv(o.kappa, o.mu, false, o.kappa);
        LQCD_K(launch_dslash(64, o.recon, false, RED_NONE, d, o.nrhs, o.dcfg, o.s));
    }
    // ||b - M x||^2, and with eo its even half, which is ||bhat - Mhat x_e||^2
    // once x_o has been reconstructed from x_e
    LQCD_K(o.full_M(xc, nullptr, false, -1.0, bc, RED_NORM, FIN_TRUE_RR, PRED_ALWAYS, nullptr, -1, -1, -1,
                    eo ? FIN_EO_RR : 0));
    return LQCD_OK;
}

// One CGNR system: plain FP64 (even-odd or full lattice) or mixed precision
// with FP64 reliable updates (even-odd).  setup / start / iter / finish
// enqueue the kernels of each phase, so one system can be driven on its own
// and several can be recorded and replayed as batched launches.
struct CgSystem {
    const lqcd_solve_params* prm = nullptr;
    SolverPlan sp;
    Op o, lo;
    bool eo = true, mixed = false;
    int nrhs = 1, nsub = 1;
    int64_t pb = 0, fb = 0;
    char* bc = nullptr;
    char* xc = nullptr;
    void *r = nullptr, *p = nullptr, *w = nullptr, *z = nullptr, *t = nullptr, *bhat = nullptr;  // FP64
    void *t64 = nullptr, *xl = nullptr, *rl = nullptr, *pl = nullptr, *wl = nullptr, *zl = nullptr, *tl = nullptr;

    int init(const Geom& g, const lqcd_op* opi, const void* U, const void* b, void* x, const lqcd_solve_params* prm_,
             const SolverPlan& plan, hipStream_t s)
    {
        prm = prm_;
        sp = plan;
        eo = prm->eo != 0;
        mixed = prm->inner_prec != 64;
        nrhs = prm->nrhs;
        nsub = eo ? 1 : 2;
        o.g = g;
        o.prec = 64;
        o.recon = opi->recon;
        o.U = U;
        o.kappa = opi->kappa;
        o.mu = opi->mu;
        o.nrhs = nrhs;
        o.pb = parity_bytes(g, 64);
        o.s = s;
        o.rs = sp.rs;
        o.tune();
        pb = o.pb;
        fb = 2 * pb;
        bc = static_cast<char*>(const_cast<void*>(b));
        xc = static_cast<char*>(x);
        r = sp.v[0];
        if (!mixed) {
            p = sp.v[1];
            w = sp.v[2];
            z = sp.v[3];
            t = eo ? sp.v[4] : nullptr;
            bhat = eo ? sp.v[5] : nullptr;
        } else {
            t64 = sp.v[1];
            bhat = sp.v[2];
            lo = o;
            lo.prec = prm->inner_prec;
            lo.recon = prm->inner_recon;
            lo.U = sp.Ulo;
            lo.pb = parity_bytes(g, lo.prec);
            lo.tune();
            xl = sp.lo[0];
            rl = sp.lo[1];
            pl = sp.lo[2];
            wl = sp.lo[3];
            zl = sp.lo[4];
            tl = sp.lo[5];
        }
        return LQCD_OK;
    }

    int setup(bool allow_fallback = false)
    {
        int rc = solver_setup(o, prm, eo, mixed, bc, xc, bhat, mixed ? t64 : t, allow_fallback);
        if (rc) return rc;
        if (mixed) LQCD_K(launch_convert_gauge(lo.prec, lo.recon, o.g, o.U, o.recon, sp.Ulo, o.s));
        return LQCD_OK;
    }

    // Continue at FP32 inner storage: the low-precision x of every right-hand
    // side is folded into the FP64 x, the inner links are rebuilt at FP32
    // (the workspace was planned for FP32 inner fields), and the next start()
    // begins from the FP64 residual.
    int fall_back_to_fp32()
    {
        LQCD_K(fold(PRED_ALWAYS));
        lo.prec = 32;
        lo.pb = parity_bytes(o.g, 32);
        lo.tune();
        LQCD_K(launch_convert_gauge(lo.prec, lo.recon, o.g, o.U, o.recon, sp.Ulo, o.s));
        return LQCD_OK;
    }

    // x_e / x as the first operand of a BLAS step (full field stride)
    hipError_t blas_x(int op, int pred, int fin, void* X, void* Y, void* Z, void* W) const
    {
        BlasArgs a = o.blas_base(nsub);
        a.pred = pred;
        a.x = X;
        a.y = Y;
        a.z = Z;
        a.w = W;
        a.st_x = fb;
        a.r.fin = fin;
        return launch_blas(64, op, a, nrhs, o.bcfg, o.s);
    }
    // r = rhs - Op x (rhs = bhat for even-odd, b for the full lattice), FP64
    hipError_t residual(void* out, int red, int fin, int pred) const
    {
        if (eo) return o.schur(xc, out, mixed ? t64 : t, false, -1.0, bhat, red, fin, pred, nullptr, fb, pb);
        return o.full_M(xc, out, false, -1.0, bc, red, fin, pred);
    }
    hipError_t apply(const void* in, void* out, bool dag, int red, int fin, int pred) const
    {
        if (eo) return o.schur(in, out, t, dag, 1.0, nullptr, red, fin, pred);
        return o.full_M(in, out, dag, 1.0, nullptr, red, fin, pred);
    }
    hipError_t to_low(void* dst, const void* src, int pred) const
    {
        ConvertArgs c{};
        c.Vh = o.g.Vh;
        c.S = o.g.S;
        c.nsub = 1;
        c.dst = dst;
        c.src = const_cast<void*>(src);
        c.rhs_stride_dst = lo.pb;
        c.rhs_stride_src = pb;
        c.pred = pred;
        c.ctl = sp.rs.ctl;
        return launch_convert(lo.prec, 64, c, nrhs, o.s);
    }
    hipError_t fold(int pred) const  // x_e += x_low ; x_low = 0
    {
        ConvertArgs c{};
        c.Vh = o.g.Vh;
        c.S = o.g.S;
        c.nsub = 1;
        c.dst = xc;
        c.src = xl;
        c.rhs_stride_dst = fb;
        c.rhs_stride_src = lo.pb;
        c.accumulate = 1;
        c.zero_src = 1;
        c.pred = pred;
        c.ctl = sp.rs.ctl;
        return launch_convert(64, lo.prec, c, nrhs, o.s);
    }

    int start()
    {
        if (!mixed) {
            // r = rhs - Op x ; z = Op^+ r ; zz ; p = z
            LQCD_K(residual(r, RED_NONE, FIN_STORE, PRED_ACTIVE));
            LQCD_K(apply(r, z, true, RED_NORM, FIN_CG_ZZ, PRED_ACTIVE));
            LQCD_K(o.blas(BLAS_COPY, nsub, PRED_ACTIVE, FIN_STORE, z, p));
            return LQCD_OK;
        }
        // r = bhat - Mhat x (FP64) ; rr_max ; r_low ; x_low = 0 ; z = Mhat^+ r_low ; p = z
        LQCD_K(residual(r, RED_NORM, FIN_RR_INIT, PRED_ACTIVE));
        LQCD_K(to_low(rl, r, PRED_ACTIVE));
        LQCD_K(lo.blas(BLAS_ZERO, 1, PRED_ACTIVE, FIN_STORE, nullptr, xl));
        LQCD_K(lo.schur(rl, zl, tl, true, 1.0, nullptr, RED_NORM, FIN_CG_ZZ, PRED_ACTIVE));
        LQCD_K(lo.blas(BLAS_COPY, 1, PRED_ACTIVE, FIN_STORE, zl, pl));
        return LQCD_OK;
    }

    int iter()
    {
        if (!mixed) {
            LQCD_K(apply(p, w, false, RED_NORM, FIN_CG_ALPHA, PRED_ACTIVE));
            LQCD_K(blas_x(BLAS_CG_XR, PRED_ACTIVE, FIN_CG_RR, xc, p, r, w));
            LQCD_K(apply(r, z, true, RED_NORM, FIN_CG_BETA, PRED_ACTIVE));
            LQCD_K(o.blas(BLAS_CG_P, nsub, PRED_ACTIVE, FIN_STORE, nullptr, p, z));
            return LQCD_OK;
        }
        LQCD_K(lo.schur(pl, wl, tl, false, 1.0, nullptr, RED_NORM, FIN_CG_ALPHA, PRED_ACTIVE));
        LQCD_K(lo.blas(BLAS_CG_XR, 1, PRED_ACTIVE, FIN_CG_RR, xl, pl, rl, wl));
        // reliable update (runs only when FIN_CG_RR requested it)
        LQCD_K(fold(PRED_UPDATE));
        LQCD_K(residual(r, RED_NORM, FIN_RU_RR, PRED_UPDATE));
        LQCD_K(to_low(rl, r, PRED_UPDATE));
        LQCD_K(lo.schur(rl, zl, tl, true, 1.0, nullptr, RED_NORM, FIN_CG_BETA, PRED_ACTIVE));
        LQCD_K(lo.blas(BLAS_CG_P, 1, PRED_ACTIVE, FIN_STORE, nullptr, pl, zl));
        return LQCD_OK;
    }

    int finish()
    {
        if (mixed) LQCD_K(fold(PRED_ALWAYS));
        return solver_finish(o, eo, bc, xc);
    }
};

int validate_solve(const lqcd_geom* geom, const lqcd_op* opi, const void* U, const void* b, void* x,
                   const lqcd_solve_params* prm, const void* info, int method, Geom* g)
{
    int rc = make_geom(geom, g);
    if (rc) return rc;
    if ((rc = check_op(opi))) return rc;
    if (opi->prec != 64) return set_error(LQCD_EINVAL, "solvers take FP64 fields (op->prec = 64)");
    if ((rc = check_params(prm, method))) return rc;
    if (!U || !b || !x || !info) return set_error(LQCD_EINVAL, "NULL field or info pointer");
    return LQCD_OK;
}

// The single-system solver (CGNR or BiCGStab, FP64 or mixed, eo or full lattice).
int solve(int method, const lqcd_geom* geom, const lqcd_op* opi, const void* U, const void* b, void* x,
          const lqcd_solve_params* prm, lqcd_solve_info* info, void* ws, size_t ws_bytes, void* stream)
{
    const double t0 = now_s();
    g_err[0] = 0;
    Geom g;
    int rc = validate_solve(geom, opi, U, b, x, prm, info, method, &g);
    if (rc) return rc;
    if (!ws) return set_error(LQCD_EINVAL, "workspace is NULL");
    if (prm->use_graph && !stream) return set_error(LQCD_EINVAL, "graph replay needs a non-default stream");
    if (prm->persistent) return set_error(LQCD_EUNSUPPORTED, "persistent launches are for cg_solve_batch");
    SolverPlan sp;
    plan_solver(g, opi, prm, method, ws, &sp);
    if (ws_bytes < sp.bytes)
        return set_error(LQCD_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, sp.bytes);

    const int nrhs = prm->nrhs;
    const bool eo = prm->eo != 0;
    const bool mixed = prm->inner_prec != 64;
    const int chunk = prm->check_every > 0 ? prm->check_every : 8;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<Ctl> ctl;
    int restarts = 0;

    unsigned fallbacks = 0;
    if (method == M_CG) {
        CgSystem cs;
        if ((rc = cs.init(g, opi, U, b, x, prm, sp, s))) return rc;
        if ((rc = cs.setup(true))) return rc;
        for (;;) {
            if ((rc = cs.start())) return rc;
            rc = drive(s, sp.rs.ctl, 1, nrhs, nrhs, chunk, prm->maxiter, prm->use_graph != 0,
                       [&]() -> int { return cs.iter(); });
            if (rc) return rc;
            if ((rc = read_ctls(s, sp.rs.ctl, nrhs, ctl))) return rc;
            unsigned fb = 0;
            for (int i = 0; i < nrhs; ++i)
                if (ctl[i].status == kStatusFallback) fb |= 1u << i;
            if (fb) {
                // stagnation at FP16 storage: the stalled right-hand sides
                // continue at FP32 from their current x
                if ((rc = cs.fall_back_to_fp32())) return rc;
                fallbacks |= fb;
                LQCD_K(launch_ctl_reopen(sp.rs.ctl, nrhs, fb, s, true));
                continue;
            }
            if ((rc = cs.finish())) return rc;
            if ((rc = read_ctls(s, sp.rs.ctl, nrhs, ctl))) return rc;
            const unsigned reopen = reopen_mask(ctl.data(), nrhs, prm);
            if (!reopen || restarts >= 20) break;
            ++restarts;
            LQCD_K(launch_ctl_reopen(sp.rs.ctl, nrhs, reopen, s));
        }
    } else {
        // BiCGStab: r r0 p v s t (tmp bhat)
        Op o;
        o.g = g;
        o.prec = 64;
        o.recon = opi->recon;
        o.U = U;
        o.kappa = opi->kappa;
        o.mu = opi->mu;
        o.nrhs = nrhs;
        o.pb = parity_bytes(g, 64);
        o.s = s;
        o.rs = sp.rs;
        o.tune();
        const int64_t pb = o.pb, fb = 2 * pb;
        const int nsub = eo ? 1 : 2;
        char* bc = static_cast<char*>(const_cast<void*>(b));
        char* xc = static_cast<char*>(x);
        void *r = sp.v[0], *r0 = sp.v[1], *p = sp.v[2], *v = sp.v[3], *sv = sp.v[4], *t = sp.v[5];
        void *tmp = sp.v[6], *bhat = sp.v[7];
        if (prm->bicgstab_ell == 2) {
            tmp = sp.v[7];
            bhat = sp.v[8];
        }
        if ((rc = solver_setup(o, prm, eo, false, bc, xc, bhat, tmp))) return rc;
        auto apply = [&](const void* in, void* out, int red, int fin, const void* aux) -> hipError_t {
            if (eo) return o.schur(in, out, tmp, false, 1.0, nullptr, red, fin, PRED_ACTIVE, aux);
            return o.full_M(in, out, false, 1.0, nullptr, red, fin, PRED_ACTIVE, aux);
        };
        auto start = [&]() -> int {
            if (eo) LQCD_K(o.schur(xc, r, tmp, false, -1.0, bhat, RED_NONE, FIN_STORE, PRED_ACTIVE, nullptr, fb, pb));
            else LQCD_K(o.full_M(xc, r, false, -1.0, bc, RED_NONE, FIN_STORE, PRED_ACTIVE));
            LQCD_K(o.blas(BLAS_COPY, nsub, PRED_ACTIVE, FIN_STORE, r, r0));
            LQCD_K(o.blas(BLAS_NORM_DOT, nsub, PRED_ACTIVE, FIN_BI_INIT, r, nullptr, nullptr, nullptr, nullptr, r0));
            LQCD_K(o.blas(BLAS_ZERO, nsub, PRED_ACTIVE, FIN_STORE, nullptr, p));
            LQCD_K(o.blas(BLAS_ZERO, nsub, PRED_ACTIVE, FIN_STORE, nullptr, v));
            return LQCD_OK;
        };
        auto iter = [&]() -> int {
            LQCD_K(o.blas(BLAS_BI_P, nsub, PRED_ACTIVE, FIN_STORE, nullptr, p, r, nullptr, v));
            LQCD_K(apply(p, v, RED_DOT_AUX, FIN_BI_ALPHA, r0));
            LQCD_K(o.blas(BLAS_BI_S, nsub, PRED_ACTIVE, FIN_STORE, nullptr, nullptr, r, sv, v));
            LQCD_K(apply(sv, t, RED_NORM_DS, FIN_BI_OMEGA, nullptr));
            BlasArgs a = o.blas_base(nsub);
            a.pred = PRED_ACTIVE;
            a.x = xc;
            a.y = p;
            a.z = r;
            a.w = sv;
            a.v = t;
            a.r0 = r0;
            a.st_x = fb;
            a.r.fin = FIN_BI_RHO;
            LQCD_K(launch_blas(64, BLAS_BI_XR, a, nrhs, o.bcfg, s));
            return LQCD_OK;
        };
        // BiCGStab(2) (Sleijpen and Fokkema 1993): one cycle is two BiCG
        // steps, each extending u_0.. and r_0.. by one application of the
        // operator, then the minimal-residual polynomial of degree 2 over
        // r_1, r_2 (Gram-Schmidt).  u_0 -= g1 u_1 + g2 u_2 of the polynomial
        // step is folded into the next cycle's first update of u_0.
        void *q0 = sp.v[0], *q1 = sp.v[1], *q2 = sp.v[2], *u0 = sp.v[3], *u1 = sp.v[4], *u2 = sp.v[5];
        void* rt = sp.v[6];
        auto start2 = [&]() -> int {
            if (eo) LQCD_K(o.schur(xc, q0, tmp, false, -1.0, bhat, RED_NONE, FIN_STORE, PRED_ACTIVE, nullptr, fb, pb));
            else LQCD_K(o.full_M(xc, q0, false, -1.0, bc, RED_NONE, FIN_STORE, PRED_ACTIVE));
            LQCD_K(o.blas(BLAS_COPY, nsub, PRED_ACTIVE, FIN_STORE, q0, rt));
            LQCD_K(o.blas(BLAS_NORM_DOT, nsub, PRED_ACTIVE, FIN_BL_INIT, q0, nullptr, nullptr, nullptr, nullptr, rt));
            for (void* u : {u0, u1, u2}) LQCD_K(o.blas(BLAS_ZERO, nsub, PRED_ACTIVE, FIN_STORE, nullptr, u));
            return LQCD_OK;
        };
        // the solution x (the even half of the caller's full field with eo) is strided by fb
        auto blas_x = [&](int op, int fin, void* y, void* z, void* w, void* v, const void* r0v) -> hipError_t {
            BlasArgs a = o.blas_base(nsub);
            a.pred = PRED_ACTIVE;
            a.x = xc;
            a.y = y;
            a.z = z;
            a.w = w;
            a.v = v;
            a.r0 = r0v;
            a.st_x = fb;
            a.r.fin = fin;
            return launch_blas(64, op, a, nrhs, o.bcfg, s);
        };
        auto iter2 = [&]() -> int {
            // first BiCG step: u_1 = A u_0, r_1 = A r_0
            LQCD_K(o.blas(BLAS_BL_U0, nsub, PRED_ACTIVE, FIN_STORE, nullptr, u0, q0, u1, u2));
            LQCD_K(apply(u0, u1, RED_DOT_AUX, FIN_BL_ALPHA, rt));
            LQCD_K(blas_x(BLAS_BL_XR0, FIN_STORE, u0, q0, u1, nullptr, nullptr));
            LQCD_K(apply(q0, q1, RED_DOT_AUX, FIN_BL_BETA, rt));
            // second BiCG step: u_2 = A u_1, r_2 = A r_1
            LQCD_K(o.blas(BLAS_BL_U01, nsub, PRED_ACTIVE, FIN_STORE, nullptr, u0, q0, u1, q1));
            LQCD_K(apply(u1, u2, RED_DOT_AUX, FIN_BL_ALPHA, rt));
            LQCD_K(blas_x(BLAS_BL_XR01, FIN_STORE, u0, q0, u1, q1, u2));
            LQCD_K(apply(q1, q2, RED_NONE, FIN_STORE, nullptr));
            // minimal residual over r_1, r_2
            LQCD_K(o.blas(BLAS_BL_GRAM, nsub, PRED_ACTIVE, FIN_BL_TAU, nullptr, nullptr, q0, q1, q2));
            LQCD_K(o.blas(BLAS_BL_ORTH, nsub, PRED_ACTIVE, FIN_BL_OMEGA, nullptr, nullptr, q0, q1, q2));
            LQCD_K(blas_x(BLAS_BL_MR, FIN_BL_RES, nullptr, q0, q1, q2, rt));
            return LQCD_OK;
        };
        const bool ell2 = prm->bicgstab_ell == 2;
        for (;;) {
            if ((rc = ell2 ? start2() : start())) return rc;
            if (ell2) rc = drive(s, sp.rs.ctl, 1, nrhs, nrhs, chunk, prm->maxiter, prm->use_graph != 0, iter2);
            else rc = drive(s, sp.rs.ctl, 1, nrhs, nrhs, chunk, prm->maxiter, prm->use_graph != 0, iter);
            if (rc) return rc;
            if ((rc = solver_finish(o, eo, bc, xc))) return rc;
            if ((rc = read_ctls(s, sp.rs.ctl, nrhs, ctl))) return rc;
            const unsigned reopen = reopen_mask(ctl.data(), nrhs, prm);
            if (!reopen || restarts >= 20) break;
            ++restarts;
            LQCD_K(launch_ctl_reopen(sp.rs.ctl, nrhs, reopen, s));
        }
    }

    int worst = LQCD_OK;
    fill_info(ctl.data(), nrhs, method, eo, mixed, restarts, now_s() - t0, prm, info, &worst, fallbacks);
    if (worst != LQCD_OK) set_error(worst, "solve did not converge for every right-hand side (status %d)", worst);
    return worst;
}

// ---------------------------------------------------------------------------
// Batched solves: several systems (lattices of any sizes, own kappa, mu and
// links) run the same CGNR program; each iteration's kernels are launched
// once for all systems, with per-system arguments in device tables.

constexpr size_t kStepTableBytes = 16 * 1024;  // per recorded step: arguments, offsets, finalizes of <= 16 systems
constexpr int kMaxSteps = 32;
static_assert(kMaxSteps <= kMaxPersistSteps, "the persistent program holds every recorded step");
// Polls of a grid barrier slot before the persistent kernel gives up (each
// poll sleeps ~30 ns and waits one device-coherent load: a few seconds,
// against phases of well under a millisecond).
constexpr int kPersistSpinLimit = 1 << 22;

// The persistent kernel's routine for a recorded step of all systems, or
// PR_NONE when the step is not one it runs (or a block shape it cannot).
int persist_routine(const std::vector<std::vector<Step>>& steps, size_t k)
{
    const Step& st = steps[0][k];
    for (const auto& sys : steps) {
        const Step& q = sys[k];
        if (q.kind == STEP_DSLASH && (q.d.block.x > (unsigned)kPersistThreads || q.d.a.lanes != 1)) return PR_NONE;
        if (q.kind == STEP_BLAS && q.b.block.x != (unsigned)kPersistThreads) return PR_NONE;
        if (q.kind == STEP_CONVERT && q.c.block.x != (unsigned)kPersistThreads) return PR_NONE;
    }
    if (st.kind == STEP_DSLASH) {
        const DslashPlan& d = st.d;
        if (d.kind != PLAN_WILSON || d.nr != 1 || d.lnt || (d.red != RED_NONE && d.red != RED_NORM)) return PR_NONE;
        const bool norm = d.red == RED_NORM;
        if (d.prec == 32 && d.recon == 12)
            return d.dag ? (norm ? PR_HOP32_12_D1_NORM : PR_HOP32_12_D1_NONE)
                         : (norm ? PR_HOP32_12_D0_NORM : PR_HOP32_12_D0_NONE);
        if (d.prec == 64 && d.recon == 18 && !d.dag) return norm ? PR_HOP64_18_D0_NORM : PR_HOP64_18_D0_NONE;
        return PR_NONE;
    }
    if (st.kind == STEP_BLAS) {
        if (st.b.prec != 32 || st.b.a.kind != KIND_SPINOR) return PR_NONE;
        if (st.b.op == BLAS_CG_XR) return PR_BLAS32_CG_XR;
        if (st.b.op == BLAS_CG_P) return PR_BLAS32_CG_P;
        return PR_NONE;
    }
    if (st.c.pd == 64 && st.c.ps == 32 && st.c.a.accumulate) return PR_CONV64_32_ACC;
    if (st.c.pd == 32 && st.c.ps == 64 && !st.c.a.accumulate) return PR_CONV32_64;
    return PR_NONE;
}

struct BatchLayout {
    Ctl* ctl = nullptr;               // nsys x kMaxRhs control blocks
    std::vector<SolverPlan> plans;
    char* tables = nullptr;           // kMaxSteps x kStepTableBytes
    PProgram* prog = nullptr;         // the persistent kernel's program
    unsigned* words = nullptr;        // its barrier slots [0, 2 kMaxPersistBlocks), then two flags
    size_t bytes = 0;
};

int plan_batch(int nsys, const Geom* g, const lqcd_op* ops, const lqcd_solve_params* prm, void* ws, BatchLayout* L)
{
    Arena ar{static_cast<char*>(ws), 0, 0};
    L->ctl = static_cast<Ctl*>(ar.take(sizeof(Ctl) * kMaxRhs * nsys));
    L->tables = static_cast<char*>(ar.take(kStepTableBytes * kMaxSteps));
    L->prog = static_cast<PProgram*>(ar.take(sizeof(PProgram)));
    L->words = static_cast<unsigned*>(ar.take((2 * kMaxPersistBlocks + 2) * sizeof(unsigned)));
    L->plans.resize(nsys);
    for (int s = 0; s < nsys; ++s) {
        ar.off = align_up(ar.off, 256);
        void* base = ws ? static_cast<char*>(ws) + ar.off : nullptr;
        plan_solver(g[s], &ops[s], prm, M_CG, base, &L->plans[s], false);
        L->plans[s].rs.ctl = L->ctl ? L->ctl + s * kMaxRhs : nullptr;
        ar.off += L->plans[s].bytes;
    }
    L->bytes = align_up(ar.off, 256);
    return LQCD_OK;
}

bool same_kernel(const Step& a, const Step& b)
{
    if (a.kind != b.kind) return false;
    if (a.kind == STEP_DSLASH)
        return a.d.kind == b.d.kind && a.d.prec == b.d.prec && a.d.recon == b.d.recon && a.d.nr == b.d.nr &&
               a.d.lnt == b.d.lnt && a.d.red == b.d.red &&
               a.d.dag == b.d.dag && a.d.a.nrhs == b.d.a.nrhs && a.d.grid.y == b.d.grid.y;
    if (a.kind == STEP_BLAS)
        return a.b.prec == b.b.prec && a.b.op == b.b.op && a.b.nrhs == b.b.nrhs && a.b.block.x == b.b.block.x;
    return a.c.pd == b.c.pd && a.c.ps == b.c.ps && a.c.a.accumulate == b.c.a.accumulate && a.c.grid.y == b.c.grid.y;
}

// The recorded iteration of every system, zipped into batched launches.
struct BatchProgram {
    int nsys = 0;
    std::vector<std::vector<Step>> steps;  // [system][step]
    std::vector<const char*> tab, offs, fin;  // device tables per step
    std::vector<int> total;                   // padded blocks per step

    int build(const std::vector<Recorder>& rec, char* dev_tables, hipStream_t s)
    {
        nsys = (int)rec.size();
        const size_t nst = rec[0].steps.size();
        if (nst > (size_t)kMaxSteps) return set_error(LQCD_EINVAL, "iteration has too many steps to batch");
        steps.assign(nsys, {});
        for (int i = 0; i < nsys; ++i) {
            if (rec[i].steps.size() != nst) return set_error(LQCD_EINVAL, "systems recorded different programs");
            steps[i] = rec[i].steps;
        }
        std::vector<char> host(kStepTableBytes * nst, 0);
        tab.resize(nst);
        offs.resize(nst);
        fin.resize(nst);
        total.resize(nst);
        for (size_t k = 0; k < nst; ++k) {
            for (int i = 1; i < nsys; ++i)
                if (!same_kernel(steps[0][k], steps[i][k])) return set_error(LQCD_EINVAL, "systems disagree at step %zu", k);
            char* h = host.data() + k * kStepTableBytes;
            size_t argsz = 0;
            const int kind = steps[0][k].kind;
            argsz = kind == STEP_DSLASH ? sizeof(DslashArgs) : kind == STEP_BLAS ? sizeof(BlasArgs) : sizeof(ConvertArgs);
            const size_t off_offs = align_up(argsz * nsys, 256);
            const size_t off_fin = align_up(off_offs + sizeof(int) * (nsys + 1), 256);
            if (off_fin + sizeof(FinArgs) * nsys > kStepTableBytes) return set_error(LQCD_EINVAL, "batch tables too large");
            int* o = reinterpret_cast<int*>(h + off_offs);
            FinArgs* f = reinterpret_cast<FinArgs*>(h + off_fin);
            int acc = 0;
            for (int i = 0; i < nsys; ++i) {
                const Step& st = steps[i][k];
                o[i] = acc;
                int gx = 0;
                if (kind == STEP_DSLASH) {
                    std::memcpy(h + i * argsz, &st.d.a, argsz);
                    gx = (int)st.d.grid.x;
                    f[i] = FinArgs{st.d.a.r.partials, st.d.slots, st.d.a.r.fin, st.d.a.ctl, st.d.a.pred};
                } else if (kind == STEP_BLAS) {
                    std::memcpy(h + i * argsz, &st.b.a, argsz);
                    gx = (int)st.b.grid.x;
                    f[i] = FinArgs{st.b.a.r.partials, st.b.slots, st.b.a.r.fin, st.b.a.ctl, st.b.a.pred};
                } else {
                    std::memcpy(h + i * argsz, &st.c.a, argsz);
                    gx = (int)st.c.grid.x;
                }
                acc += (gx + 7) / 8 * 8;  // each system starts on a multiple of 8 (XCD remap)
            }
            o[nsys] = acc;
            total[k] = acc;
            const char* d = dev_tables + k * kStepTableBytes;
            tab[k] = d;
            offs[k] = d + off_offs;
            fin[k] = d + off_fin;
        }
        LQCD_HIP(hipMemcpyAsync(dev_tables, host.data(), host.size(), hipMemcpyHostToDevice, s));
        LQCD_HIP(hipStreamSynchronize(s));
        return LQCD_OK;
    }

    // The recorded iteration as the persistent kernel's program (host copy);
    // false when some step is not one the kernel runs.
    bool persistent_program(PProgram* P) const
    {
        const size_t nst = steps[0].size();
        *P = PProgram{};
        P->nsteps = (int)nst;
        for (size_t k = 0; k < nst; ++k) {
            const int r = persist_routine(steps, k);
            if (r == PR_NONE) return false;
            const Step& st = steps[0][k];
            PStep& ps = P->step[k];
            ps.routine = r;
            ps.total = total[k];
            unsigned gy = 1;
            int nfin = 0;
            for (int i = 0; i < nsys; ++i) {
                const Step& q = steps[i][k];
                const unsigned y = q.kind == STEP_DSLASH ? q.d.grid.y : q.kind == STEP_BLAS ? q.b.grid.y : q.c.grid.y;
                gy = y > gy ? y : gy;
            }
            if (st.kind == STEP_DSLASH) nfin = st.d.nfin;
            else if (st.kind == STEP_BLAS) nfin = st.b.nfin;
            ps.gy = (int)gy;
            ps.nfin = nfin;
            ps.pred = st.kind == STEP_DSLASH ? st.d.a.pred : st.kind == STEP_BLAS ? st.b.a.pred : st.c.a.pred;
            for (int i = 1; i < nsys; ++i) {
                const Step& q = steps[i][k];
                const int pi = q.kind == STEP_DSLASH ? q.d.a.pred : q.kind == STEP_BLAS ? q.b.a.pred : q.c.a.pred;
                if (pi != ps.pred) return false;
            }
            ps.tab = tab[k];
            ps.offs = reinterpret_cast<const int*>(offs[k]);
            ps.fin = reinterpret_cast<const FinArgs*>(fin[k]);
        }
        return true;
    }

    int run(hipStream_t s) const
    {
        const size_t nst = steps[0].size();
        std::vector<DslashPlan> dp(nsys);
        std::vector<BlasPlan> bp(nsys);
        std::vector<ConvertPlan> cp(nsys);
        for (size_t k = 0; k < nst; ++k) {
            const int kind = steps[0][k].kind;
            hipError_t e;
            if (kind == STEP_DSLASH) {
                for (int i = 0; i < nsys; ++i) dp[i] = steps[i][k].d;
                e = exec_dslash_batch(dp.data(), nsys, reinterpret_cast<const DslashArgs*>(tab[k]),
                                      reinterpret_cast<const int*>(offs[k]), total[k],
                                      reinterpret_cast<const FinArgs*>(fin[k]), s);
            } else if (kind == STEP_BLAS) {
                for (int i = 0; i < nsys; ++i) bp[i] = steps[i][k].b;
                e = exec_blas_batch(bp.data(), nsys, reinterpret_cast<const BlasArgs*>(tab[k]),
                                    reinterpret_cast<const int*>(offs[k]), total[k],
                                    reinterpret_cast<const FinArgs*>(fin[k]), s);
            } else {
                for (int i = 0; i < nsys; ++i) cp[i] = steps[i][k].c;
                e = exec_convert_batch(cp.data(), nsys, reinterpret_cast<const ConvertArgs*>(tab[k]),
                                       reinterpret_cast<const int*>(offs[k]), total[k], s);
            }
            if (e != hipSuccess) return set_error(LQCD_EHIP, "batched launch failed: %s", hipGetErrorString(e));
        }
        return LQCD_OK;
    }
};

int solve_batch(int nsys, const lqcd_geom* geoms, const lqcd_op* ops, const void* const* U, const void* const* b,
                void* const* x, const lqcd_solve_params* prm, lqcd_solve_info* info, void* ws, size_t ws_bytes,
                void* stream)
{
    const double t0 = now_s();
    g_err[0] = 0;
    if (nsys < 1 || nsys > kMaxSys) return set_error(LQCD_EINVAL, "nsys %d not in [1, %d]", nsys, kMaxSys);
    if (!geoms || !ops || !U || !b || !x || !info) return set_error(LQCD_EINVAL, "NULL array argument");
    std::vector<Geom> g(nsys);
    int rc;
    for (int s = 0; s < nsys; ++s)
        if ((rc = validate_solve(&geoms[s], &ops[s], U[s], b[s], x[s], prm, info, M_CG, &g[s]))) return rc;
    if (!ws) return set_error(LQCD_EINVAL, "workspace is NULL");
    if (prm->use_graph && !stream) return set_error(LQCD_EINVAL, "graph replay needs a non-default stream");
    if (prm->persistent) {
        bool ok = prm->nrhs >= 2 && prm->inner_prec == 32 && prm->inner_recon == 12 && prm->eo;
        for (int s = 0; s < nsys; ++s) ok = ok && ops[s].recon == 18;
        if (!ok)
            return set_error(LQCD_EUNSUPPORTED, "the persistent batched solve runs the even-odd mixed CGNR with FP32/12 "
                                                "inner and 18-real FP64 outer hops on nrhs >= 2 right-hand sides");
    }
    BatchLayout L;
    plan_batch(nsys, g.data(), ops, prm, ws, &L);
    if (ws_bytes < L.bytes) return set_error(LQCD_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nrhs = prm->nrhs;
    const int chunk = prm->check_every > 0 ? prm->check_every : 8;

    std::vector<CgSystem> sys(nsys);
    for (int s = 0; s < nsys; ++s) {
        if ((rc = sys[s].init(g[s], &ops[s], U[s], b[s], x[s], prm, L.plans[s], st))) return rc;
        if ((rc = sys[s].setup())) return rc;
    }
    // record one iteration per system and zip the recordings into batched launches
    std::vector<Recorder> rec(nsys);
    for (int s = 0; s < nsys; ++s) {
        set_recorder(&rec[s]);
        rc = sys[s].iter();
        set_recorder(nullptr);
        if (rc) return rc;
    }
    BatchProgram prog;
    if ((rc = prog.build(rec, L.tables, st))) return rc;

    // One persistent cooperative launch per start: the program, the grid
    // (the blocks the device keeps resident) and the barrier words.
    int pgrid = 0, launches = 0;
    PProgram P{};
    if (prm->persistent) {
        if (nrhs < 2 || !prog.persistent_program(&P))
            return set_error(LQCD_EUNSUPPORTED, "the persistent batched solve runs the mixed CGNR with FP32/12 inner "
                                                "and 18-real FP64 outer hops on nrhs >= 2 right-hand sides");
        hipError_t e = persistent_grid(&pgrid);
        if (e != hipSuccess) return set_error(LQCD_EUNSUPPORTED, "no cooperative launch on this device: %s",
                                              hipGetErrorString(e));
        // no more blocks than the largest phase has (the others would only
        // wait at every barrier) nor than the barrier has slots for
        int64_t widest = 1;
        for (int k = 0; k < P.nsteps; ++k) widest = std::max<int64_t>(widest, (int64_t)P.step[k].total * P.step[k].gy);
        pgrid = (int)std::min<int64_t>({(int64_t)pgrid, widest, (int64_t)kMaxPersistBlocks});
        P.nsys = nsys;
        P.nrhs = nrhs;
        P.ctl_stride = kMaxRhs;
        P.ctl = L.ctl;
        P.max_iter = prm->maxiter + 1;
        P.spin_limit = kPersistSpinLimit;
        P.bar = L.words;
        P.flag = reinterpret_cast<int*>(L.words + 2 * kMaxPersistBlocks);
        LQCD_HIP(hipMemcpyAsync(L.prog, &P, sizeof(PProgram), hipMemcpyHostToDevice, st));
        LQCD_HIP(hipStreamSynchronize(st));
    }

    // the captured persistent launch (use_graph), destroyed on every way out
    struct GraphHold {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        ~GraphHold()
        {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
        }
    } pgraph;
    std::vector<Ctl> ctl;
    int restarts = 0;
    for (;;) {
        for (int s = 0; s < nsys; ++s)
            if ((rc = sys[s].start())) return rc;
        if (prm->persistent) {
            // barrier slots zero and the give-up word set for persistent = 2
            // (a kernel), then the cooperative launch; with use_graph both
            // are captured once and replayed at every start
            const int give_up = prm->persistent == 2 ? 1 : 0;
            if (prm->use_graph) {
                if (!pgraph.exec) {
                    LQCD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                    hipError_t e1 = launch_persist_reset(L.words, 2 * kMaxPersistBlocks, give_up, st);
                    if (e1 == hipSuccess) e1 = launch_batch_persistent(L.prog, pgrid, st);
                    hipGraph_t gph = nullptr;
                    const hipError_t e2 = hipStreamEndCapture(st, &gph);
                    pgraph.graph = gph;
                    if (e1 != hipSuccess || e2 != hipSuccess)
                        return set_error(LQCD_EHIP, "capture of the persistent launch failed: %s",
                                         hipGetErrorString(e1 != hipSuccess ? e1 : e2));
                    LQCD_HIP(hipGraphInstantiate(&pgraph.exec, pgraph.graph, nullptr, nullptr, 0));
                }
                LQCD_HIP(hipGraphLaunch(pgraph.exec, st));
            } else {
                LQCD_HIP(launch_persist_reset(L.words, 2 * kMaxPersistBlocks, give_up, st));
                LQCD_HIP(launch_batch_persistent(L.prog, pgrid, st));
            }
            ++launches;
            unsigned back[2] = {0u, 0u};
            LQCD_HIP(hipMemcpyAsync(back, L.words + 2 * kMaxPersistBlocks, sizeof(back), hipMemcpyDeviceToHost, st));
            LQCD_HIP(hipStreamSynchronize(st));
            if (back[1] != 0u)
                return set_error(LQCD_EHIP, "persistent batched solve: a grid barrier gave up (%s)",
                                 prm->persistent == 2 ? "give-up word set at launch" : "wait beyond the spin limit");
        } else {
            rc = drive(st, L.ctl, nsys, kMaxRhs, nrhs, chunk, prm->maxiter, prm->use_graph != 0,
                       [&]() -> int { return prog.run(st); });
            if (rc) return rc;
        }
        for (int s = 0; s < nsys; ++s)
            if ((rc = sys[s].finish())) return rc;
        if ((rc = read_ctls(st, L.ctl, nsys * kMaxRhs, ctl))) return rc;
        bool any = false;
        std::vector<unsigned> masks(nsys);
        for (int s = 0; s < nsys; ++s) any = (masks[s] = reopen_mask(ctl.data() + s * kMaxRhs, nrhs, prm)) || any;
        if (!any || restarts >= 20) break;
        ++restarts;
        for (int s = 0; s < nsys; ++s)
            if (masks[s]) LQCD_K(launch_ctl_reopen(L.ctl + s * kMaxRhs, nrhs, masks[s], st));
    }
    int worst = LQCD_OK;
    const double secs = now_s() - t0;
    for (int s = 0; s < nsys; ++s)
        fill_info(ctl.data() + s * kMaxRhs, nrhs, M_CG, prm->eo != 0, prm->inner_prec != 64, restarts, secs, prm,
                  info + s * nrhs, &worst);
    for (int i = 0; i < nsys * nrhs; ++i) info[i].persistent_launches = launches;
    if (worst != LQCD_OK) set_error(worst, "batched solve did not converge for every system (status %d)", worst);
    return worst;
}


// Autotuner of a batch: the inner hop's launch shape timed inside the batched
// CGNR iteration itself (every system, its volume, its right-hand sides),
// since the shape that is fastest for one lattice alone need not be for the
// mix.  For each candidate the systems are set up from scratch, one iteration
// is recorded and zipped exactly as cg_solve_batch does, started, run once to
// warm up and then timed over `iters` iterations with HIP events.
int autotune_batch(int nsys, const lqcd_geom* geoms, const lqcd_op* ops, const void* const* U, const void* const* b,
                   void* const* x, const lqcd_solve_params* prm, void* ws, size_t ws_bytes, int iters, void* stream,
                   lqcd_launch* best, double* best_us)
{
    g_err[0] = 0;
    if (nsys < 1 || nsys > kMaxSys) return set_error(LQCD_EINVAL, "nsys %d not in [1, %d]", nsys, kMaxSys);
    if (!geoms || !ops || !U || !b || !x) return set_error(LQCD_EINVAL, "NULL array argument");
    if (iters < 1 || iters > 1000) return set_error(LQCD_EINVAL, "iters %d not in [1, 1000]", iters);
    std::vector<lqcd_solve_info> scratch_info(kMaxRhs);
    std::vector<Geom> g(nsys);
    int rc;
    for (int s = 0; s < nsys; ++s)
        if ((rc = validate_solve(&geoms[s], &ops[s], U[s], b[s], x[s], prm, scratch_info.data(), M_CG, &g[s])))
            return rc;
    if (!ws) return set_error(LQCD_EINVAL, "workspace is NULL");
    if (prm->persistent) return set_error(LQCD_EINVAL, "tune with persistent = 0 (the batched launches)");
    BatchLayout L;
    plan_batch(nsys, g.data(), ops, prm, ws, &L);
    if (ws_bytes < L.bytes) return set_error(LQCD_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nrhs = prm->nrhs;
    const int prec = prm->inner_prec;
    const int family = nrhs > 1 ? LQCD_KERNEL_DSLASH_RHS : LQCD_KERNEL_DSLASH;
    const Launch orig = launch_for(family, prec);
    std::vector<Launch> cand;
    for (int blk : {128, 192, 256}) {
        Launch c = orig;
        c.block = blk;
        c.rhs_lanes = 1;
        if (nrhs > 1) {
            c.order = orig.order < 1 ? 1 : orig.order;
            c.swizzle = 1;
            const int tg[7][2] = {{1, 0}, {1, 2}, {1, 4}, {1, 8}, {2, 0}, {2, 2}, {2, 4}};
            for (const auto& t : tg) {
                if (dslash_rhs_tile(prec, t[0], nrhs) != t[0] || t[0] * t[1] > 2 * nrhs) continue;
                c.rhs_tile = t[0];
                c.rhs_group = t[1];
                cand.push_back(c);
            }
        } else {
            for (int order : {0, 1})
                for (int swz : {0, 1}) {
                    c.order = order;
                    c.swizzle = swz;
                    cand.push_back(c);
                }
        }
    }
    auto install = [&](const Launch& l) {
        std::lock_guard<std::mutex> lk(g_launch_mu);
        g_launch[family][prec_slot(prec)] = l;
    };
    hipEvent_t e0, e1;
    LQCD_HIP(hipEventCreate(&e0));
    LQCD_HIP(hipEventCreate(&e1));
    Launch win = orig;
    float win_ms = -1.f;
    int result = LQCD_OK;
    for (const Launch& c : cand) {
        install(c);
        std::vector<CgSystem> sys(nsys);
        for (int s = 0; s < nsys && !result; ++s) {
            if ((result = sys[s].init(g[s], &ops[s], U[s], b[s], x[s], prm, L.plans[s], st))) break;
            result = sys[s].setup();
        }
        std::vector<Recorder> rec(nsys);
        for (int s = 0; s < nsys && !result; ++s) {
            set_recorder(&rec[s]);
            result = sys[s].iter();
            set_recorder(nullptr);
        }
        BatchProgram prog;
        if (!result) result = prog.build(rec, L.tables, st);
        for (int s = 0; s < nsys && !result; ++s) result = sys[s].start();
        if (!result) result = prog.run(st);
        if (result) break;
        hipError_t e = hipEventRecord(e0, st);
        for (int i = 0; i < iters && e == hipSuccess && !result; ++i) result = prog.run(st);
        if (result) break;
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            result = set_error(LQCD_EHIP, "batch autotune: %s", hipGetErrorString(e));
            break;
        }
        if (win_ms < 0.f || ms < win_ms) {
            win_ms = ms;
            win = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    install(result ? orig : win);
    if (result) return result;
    if (best) {
        best->block = win.block;
        best->swizzle = win.swizzle;
        best->order = win.order;
        best->rhs_tile = win.rhs_tile;
        best->rhs_group = win.rhs_group;
        best->ygroup = win.ygroup;
        best->rhs_lanes = win.rhs_lanes;
    }
    if (best_us) *best_us = 1e3 * win_ms / iters;
    return LQCD_OK;
}

// Times the even-odd hop of one kernel family (launch(cfg) enqueues one hop
// with launch shape cfg) in the 32 shapes {memory order, row tiles with y-chunk
// groups of 1, 2, 3} x {XCD remap off, on} x block {64, 128, 192, 256} with
// HIP events, keeps the
// fastest in the process-wide table (the right-hand-side tile and group of
// the family are kept: they only matter for several right-hand sides) and
// reports it.  Synchronises the stream.
template <class F>
int autotune_hop(int kernel, int prec, int recon, const int L[4], int reps, hipStream_t s, lqcd_launch* best,
                 double* best_us, F&& launch)
{
    hipEvent_t e0, e1;
    LQCD_HIP(hipEventCreate(&e0));
    LQCD_HIP(hipEventCreate(&e1));
    Launch win{};
    float win_ms = 0.f;
    bool have = false;
    int result = LQCD_OK;
    const int ygroups[3] = {1, 2, 3};
    for (int order = 0; order < 2 && !result; ++order)
        for (int yi = 0; yi < (order ? 3 : 1) && !result; ++yi)
        for (int sw = 0; sw < 2 && !result; ++sw)
            for (int blk = 64; blk <= 256 && !result; blk += 64) {
                const Launch cfg{blk, sw, order, 1, 0, ygroups[yi]};
                hipError_t e = hipSuccess;
                for (int i = 0; i < 2 && e == hipSuccess; ++i) e = launch(cfg);
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch(cfg);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    result = set_error(LQCD_EHIP, "autotune: %s", hipGetErrorString(e));
                    break;
                }
                if (!have || ms < win_ms) {
                    have = true;
                    win_ms = ms;
                    win = cfg;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result) return result;
    {
        std::lock_guard<std::mutex> lk(g_launch_mu);
        Launch& slot = g_launch[kernel][prec_slot(prec)];
        win.rhs_tile = slot.rhs_tile;
        win.rhs_group = slot.rhs_group;
        win.rhs_lanes = slot.rhs_lanes;
        slot = win;
    }
    tune_record(kernel, prec, recon, L, 1, win, 1e3 * win_ms / reps);
    if (best) {
        best->block = win.block;
        best->swizzle = win.swizzle;
        best->order = win.order;
        best->rhs_tile = win.rhs_tile;
        best->rhs_group = win.rhs_group;
        best->ygroup = win.ygroup;
        best->rhs_lanes = win.rhs_lanes;
    }
    if (best_us) *best_us = 1e3 * win_ms / reps;
    return LQCD_OK;
}

// ---------------------------------------------------------------------------
// Staggered fermions: the operator compositions and the (multi-shift) CG.

int check_stag_op(const lqcd_stag_op* op)
{
    if (!op) return set_error(LQCD_EINVAL, "op is NULL");
    int rc = check_prec(op->prec, op->recon);
    if (rc) return rc;
    if (!std::isfinite(op->mass)) return set_error(LQCD_EINVAL, "mass must be finite");
    return LQCD_OK;
}

int64_t colour_bytes(const Geom& g, int prec) { return colour_parity_bytes(prec, g.S); }

// The staggered operator bound to a gauge field, a precision and a stream.
// hop() is the even-odd kernel with c = 1/2 giving D; the compositions:
//   D_{p,1-p} in        : hop(p, in, out, c = 1/2)
//   (N + s) in, even    : t = D_oe in; out = (m^2 + s) in - D_eo t
//   M in, full lattice  : out = m in + D in   (M^+ : m in - D in)
struct StagOp {
    Geom g;
    int prec = 64, recon = 18;
    const void* U = nullptr;
    double mass = 0;
    int nrhs = 1;
    int64_t pb = 0;  // bytes of one parity colour field at prec
    hipStream_t s = nullptr;
    RedScratch rs;
    Launch dcfg, bcfg;

    void tune()
    {
        dcfg = launch_for(LQCD_KERNEL_STAG, prec, recon, g, nrhs);
        bcfg = launch_for(LQCD_KERNEL_BLAS, prec);
    }

    DslashArgs base(Ctl* ctl) const
    {
        DslashArgs a{};
        a.g = g;
        a.U = U;
        a.st_in = a.st_out = a.st_site = a.st_add = a.st_aux = pb;
        a.par_bytes = pb;
        a.r.partials = rs.partials;
        a.r.capacity = rs.capacity;
        a.ctl = ctl;
        return a;
    }

    // out(parity p) = add + a * site + c * sum_mu eta_mu [U in(x+mu) - U^+ in(x-mu)]
    hipError_t hop(int p, const void* in, void* out, double c, const void* site, double a, const void* add, int red,
                   int fin, int pred, Ctl* ctl) const
    {
        DslashArgs d = base(ctl);
        d.parity = p;
        d.pred = pred;
        d.in = in;
        d.out = out;
        d.site = site;
        d.add = add;
        d.a = coef_real(a);
        d.c = coef_real(c);
        d.r.fin = fin;
        return launch_stag(prec, recon, red, d, nrhs, dcfg, s);
    }

    // out = add + sgn (N + shift) in on even fields; tmp: an odd field.
    hipError_t normal(const void* in, void* out, void* tmp, double shift, double sgn, const void* add, int red, int fin,
                      int pred, Ctl* ctl) const
    {
        hipError_t e = hop(1, in, tmp, 0.5, nullptr, 0.0, nullptr, RED_NONE, FIN_STORE, pred, ctl);
        if (e != hipSuccess) return e;
        return hop(0, tmp, out, -0.5 * sgn, in, sgn * (mass * mass + shift), add, red, fin, pred, ctl);
    }

    // out = add + sgn M in (M^+ for dag) on full-lattice fields, one launch.
    hipError_t full_M(const void* in, void* out, bool dag, double sgn, const void* add, int red, int fin, int pred,
                      Ctl* ctl) const
    {
        DslashArgs d = base(ctl);
        d.full = 1;
        d.pred = pred;
        d.in = in;
        d.site = in;
        d.out = out;
        d.add = add;
        d.st_in = d.st_site = d.st_out = d.st_add = 2 * pb;
        d.a = coef_real(sgn * mass);
        d.c = coef_real((dag ? -0.5 : 0.5) * sgn);
        d.r.fin = fin;
        return launch_stag(prec, recon, red, d, nrhs, dcfg, s);
    }

    hipError_t blas(int op, int n, int pred, int fin, Ctl* ctl, void* x, int64_t st_x, void* y = nullptr,
                    int64_t st_y = 0, void* z = nullptr, int64_t st_z = 0, void* w = nullptr, int64_t st_w = 0,
                    int nsub = 1) const
    {
        BlasArgs a{};
        a.kind = KIND_COLOUR;
        a.Vh = g.Vh;
        a.S = g.S;
        a.nsub = nsub;
        a.sub_stride = pb;
        a.pred = pred;
        a.x = x;
        a.y = y;
        a.z = z;
        a.w = w;
        a.st_x = st_x;
        a.st_y = st_y;
        a.st_z = st_z;
        a.st_w = st_w;
        a.r.partials = rs.partials;
        a.r.capacity = rs.capacity;
        a.r.fin = fin;
        a.ctl = ctl;
        return launch_blas(prec, op, a, n, bcfg, s);
    }
};

// Workspace of a staggered solve: reductions (one right-hand side), control
// blocks for up to kMaxShifts systems, then the vectors.
struct StagPlan {
    RedScratch rs;
    void* r = nullptr;     // even: residual
    void* w = nullptr;     // even: (N + s0) p
    void* t = nullptr;     // odd scratch
    void* bhat = nullptr;  // even: m b_e - D_eo b_o (CG)
    void* p = nullptr;     // nshift even fields (multi-shift) or one (CG)
    size_t bytes = 0;
};

void plan_stag(const Geom& g, int nshift, void* ws, StagPlan* sp)
{
    Arena ar{static_cast<char*>(ws), 0, 0};
    const int64_t nblk = max_blocks(g);
    sp->rs.capacity = (int)nblk;
    sp->rs.partials = static_cast<double*>(ar.take(sizeof(double) * 3 * nblk));
    sp->rs.ctl = static_cast<Ctl*>(ar.take(sizeof(Ctl) * kMaxShifts));
    const size_t pb = (size_t)colour_bytes(g, 64);
    sp->r = ar.take(pb);
    sp->w = ar.take(pb);
    sp->t = ar.take(pb);
    sp->bhat = nshift == 0 ? ar.take(pb) : nullptr;
    sp->p = ar.take(pb * (size_t)(nshift > 0 ? nshift : 1));
    sp->bytes = align_up(ar.off, 256);
}

int check_stag_params(const lqcd_solve_params* p)
{
    if (!p) return set_error(LQCD_EINVAL, "params is NULL");
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return set_error(LQCD_EINVAL, "tol must be > 0");
    if (p->maxiter < 0) return set_error(LQCD_EINVAL, "maxiter < 0");
    if (p->eo != 1) return set_error(LQCD_EUNSUPPORTED, "staggered solves are even-odd (eo = 1)");
    if (p->inner_prec != 64) return set_error(LQCD_EUNSUPPORTED, "staggered solves are FP64 (inner_prec = 64)");
    if (p->nrhs != 1) return set_error(LQCD_EUNSUPPORTED, "staggered solves take one right-hand side (nrhs = 1)");
    return LQCD_OK;
}

// The CG iteration on the base system (control block ctl + base) of the
// shifted family (N + s_i), i < n, with x_i, p_i at stride pb:
//   w = (N + s_base) p_base, alpha and every zeta_{k+1}, alpha_i  (FIN_MS_ALPHA)
//   x_i += alpha_i p_i
//   r -= alpha w, ||r||^2, beta, beta_i, zeta shift, convergence  (FIN_MS_BETA)
//   p_i = zeta_i r + beta_i p_i
int stag_ms_iter(const StagOp& o, const StagPlan& sp, char* x, int n, int base, double s_base)
{
    Ctl* ctl = sp.rs.ctl;
    char* p = static_cast<char*>(sp.p);
    const int64_t pb = o.pb;
    LQCD_K(o.normal(p + base * pb, sp.w, sp.t, s_base, 1.0, nullptr, RED_NORM_DS, FIN_MS_ALPHA, PRED_ACTIVE,
                    ctl + base));
    LQCD_K(o.blas(BLAS_MS_AXPY, n, PRED_ACTIVE, FIN_STORE, ctl, x, pb, p, pb));
    LQCD_K(o.blas(BLAS_AXMY_NORM, 1, PRED_ACTIVE, FIN_MS_BETA, ctl + base, nullptr, 0, nullptr, 0, sp.r, pb, sp.w,
                  pb));
    LQCD_K(o.blas(BLAS_MS_P, n, PRED_ACTIVE, FIN_STORE, ctl, nullptr, 0, p, pb, sp.r, 0));
    return LQCD_OK;
}

int stag_validate(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* b, void* x,
                  const lqcd_solve_params* prm, const void* info, void* ws, void* stream, Geom* g)
{
    int rc = make_geom(geom, g);
    if (rc) return rc;
    if ((rc = check_stag_op(op))) return rc;
    if (op->prec != 64) return set_error(LQCD_EINVAL, "solvers take FP64 fields (op->prec = 64)");
    if (!(op->mass > 0.0)) return set_error(LQCD_EINVAL, "the even-odd solve needs mass > 0");
    if ((rc = check_stag_params(prm))) return rc;
    if (!U || !b || !x || !info) return set_error(LQCD_EINVAL, "NULL field or info pointer");
    if (!ws) return set_error(LQCD_EINVAL, "workspace is NULL");
    if (prm->use_graph && !stream) return set_error(LQCD_EINVAL, "graph replay needs a non-default stream");
    return LQCD_OK;
}

StagOp stag_bind(const Geom& g, const lqcd_stag_op* op, const void* U, const StagPlan& sp, void* stream)
{
    StagOp o;
    o.g = g;
    o.prec = 64;
    o.recon = op->recon;
    o.U = U;
    o.mass = op->mass;
    o.nrhs = 1;
    o.pb = colour_bytes(g, 64);
    o.s = static_cast<hipStream_t>(stream);
    o.rs = sp.rs;
    o.tune();
    return o;
}

// Argument checks shared by dslash_eo_apply and its variant without allocation.
int eo_apply_check(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out,
                   int32_t out_parity, int32_t op_kind, int32_t nrhs, Geom* g)
{
    int rc = make_geom(geom, g);
    if (rc) return rc;
    if ((rc = check_op(op))) return rc;
    if (!U || !in || !out) return set_error(LQCD_EINVAL, "NULL field pointer");
    if (in == out) return set_error(LQCD_EINVAL, "in and out must not alias");
    if (out_parity != 0 && out_parity != 1) return set_error(LQCD_EINVAL, "out_parity must be 0 or 1");
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(LQCD_EINVAL, "nrhs %d not in [1, %d]", nrhs, kMaxRhs);
    if (op_kind != LQCD_OP_HOP && op_kind != LQCD_OP_SCHUR) return set_error(LQCD_EINVAL, "unknown op_kind %d", op_kind);
    if (op_kind == LQCD_OP_SCHUR && out_parity != 0)
        return set_error(LQCD_EINVAL, "the Schur complement acts on even sites (out_parity 0)");
    return LQCD_OK;
}

// The hop or Schur complement; tmp holds nrhs odd parity fields at op->prec (Schur).
int eo_apply_run(const Geom& g, const lqcd_op* op, const void* U, const void* in, void* out, int32_t out_parity,
                 int32_t op_kind, int32_t dagger, int32_t nrhs, void* tmp, void* stream)
{
    Op o;
    o.g = g;
    o.prec = op->prec;
    o.recon = op->recon;
    o.U = U;
    o.kappa = op->kappa;
    o.mu = op->mu;
    o.nrhs = nrhs;
    o.pb = parity_bytes(g, op->prec);
    o.s = static_cast<hipStream_t>(stream);
    o.tune();
    if (op_kind == LQCD_OP_HOP) {
        LQCD_K(o.hop(out_parity, in, out, dagger != 0, SpinCoef{}, nullptr, coef_real(1.0), nullptr, RED_NONE,
                     FIN_STORE, PRED_ALWAYS));
        return LQCD_OK;
    }
    LQCD_K(o.schur(in, out, tmp, dagger != 0, 1.0, nullptr, RED_NONE, FIN_STORE, PRED_ALWAYS));
    return LQCD_OK;
}

// Device memory of dslash_eo_apply_noalloc: the odd-parity temporary of the
// Schur complement lives here instead of in a caller workspace.  Each GPU the
// library runs on holds its own copy for the life of the process; every call
// on one GPU uses the same bytes (the temporary is fully rewritten by each
// call, so nothing needs clearing; calls that overlap on one GPU race).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this GPU's copy of scratch, looked up once per device
// (the host-side name of the array is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(LQCD_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    }
    if (dev < 0 || dev >= kMaxDevices) return set_error(LQCD_EUNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(LQCD_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                             hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LQCD_OK;
}

}  // namespace

extern "C" {

const char* lqcd_last_error(void) { return g_err; }

const char* lqcd_version(void) { return "lqcd-gfx950 1.0"; }

int lqcd_device_memory(int32_t device, int32_t* clock_khz, int32_t* bus_bits)
{
    if (!clock_khz || !bus_bits) return set_error(LQCD_EINVAL, "NULL output pointer");
    int c = 0, w = 0;
    hipError_t e = hipDeviceGetAttribute(&c, hipDeviceAttributeMemoryClockRate, device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&w, hipDeviceAttributeMemoryBusWidth, device);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // a failed query must not linger as the runtime's last error for later launches
        return set_error(LQCD_EHIP, "device attribute query failed: %s", hipGetErrorString(e));
    }
    *clock_khz = c;
    *bus_bits = w;
    return LQCD_OK;
}

int lqcd_field_bytes(const lqcd_geom* geom, int32_t kind, int32_t prec, int32_t recon, size_t* bytes)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if (!bytes) return set_error(LQCD_EINVAL, "bytes is NULL");
    if (kind == LQCD_FIELD_GAUGE) {
        if ((rc = check_prec(prec, recon))) return rc;
        *bytes = (size_t)gauge_bytes(g, prec, recon);
        return LQCD_OK;
    }
    if ((rc = check_prec(prec, 12))) return rc;
    if (kind == LQCD_FIELD_SPINOR_PARITY) *bytes = (size_t)parity_bytes(g, prec);
    else if (kind == LQCD_FIELD_SPINOR_FULL) *bytes = (size_t)(2 * parity_bytes(g, prec));
    else if (kind == LQCD_FIELD_COLOUR_PARITY) *bytes = (size_t)colour_bytes(g, prec);
    else if (kind == LQCD_FIELD_COLOUR_FULL) *bytes = (size_t)(2 * colour_bytes(g, prec));
    else return set_error(LQCD_EINVAL, "unknown field kind %d", kind);
    return LQCD_OK;
}

int lqcd_workspace_bytes(const lqcd_geom* geom, const lqcd_op* op, const lqcd_solve_params* params, size_t* bytes)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_op(op))) return rc;
    if (!bytes) return set_error(LQCD_EINVAL, "bytes is NULL");
    if (!params) {
        // dslash_*: reductions plus one parity field per right-hand side
        Arena ar{nullptr, 0, 0};
        RedScratch rs;
        plan_reductions(ar, g, kMaxRhs, &rs);
        ar.take((size_t)(parity_bytes(g, op->prec) * kMaxRhs));
        *bytes = align_up(ar.off, 256);
        return LQCD_OK;
    }
    size_t best = 0;
    for (int method = 0; method < 2; ++method) {
        if (params->inner_prec != 64 && method == M_BICG) continue;
        if ((rc = check_params(params, method))) return rc;
        SolverPlan sp;
        plan_solver(g, op, params, method, nullptr, &sp);
        best = sp.bytes > best ? sp.bytes : best;
    }
    *bytes = best;
    return LQCD_OK;
}

int lqcd_set_launch(int32_t kernel, int32_t prec, const lqcd_launch* cfg)
{
    if (kernel != LQCD_KERNEL_DSLASH && kernel != LQCD_KERNEL_BLAS && kernel != LQCD_KERNEL_STAG &&
        kernel != LQCD_KERNEL_DSLASH_RHS)
        return set_error(LQCD_EINVAL, "unknown kernel %d", kernel);
    const int k = prec_slot(prec);
    if (k < 0) return set_error(LQCD_EINVAL, "prec %d not in {64, 32, 16}", prec);
    if (!cfg) return set_error(LQCD_EINVAL, "cfg is NULL");
    if (cfg->block < 64 || cfg->block > 256 || cfg->block % 64)
        return set_error(LQCD_EINVAL, "block %d not in {64, 128, 192, 256}", cfg->block);
    if (cfg->swizzle != 0 && cfg->swizzle != 1) return set_error(LQCD_EINVAL, "swizzle must be 0 or 1");
    if (cfg->order < 0 || cfg->order > 64) return set_error(LQCD_EINVAL, "order must be in 0..64");
    if (cfg->order >= 1 && kernel == LQCD_KERNEL_BLAS)
        return set_error(LQCD_EINVAL, "order >= 1 applies to the hop kernels only");
    if (cfg->rhs_tile != 1 && cfg->rhs_tile != 2 && cfg->rhs_tile != 4)
        return set_error(LQCD_EINVAL, "rhs_tile %d not in {1, 2, 4}", cfg->rhs_tile);
    if (cfg->rhs_group != 0 && (cfg->rhs_group < 2 || cfg->rhs_group > 16))
        return set_error(LQCD_EINVAL, "rhs_group %d not 0 or in [2, 16]", cfg->rhs_group);
    if (cfg->ygroup < 0 || cfg->ygroup > 64) return set_error(LQCD_EINVAL, "ygroup %d not in [0, 64]", cfg->ygroup);
    if (cfg->rhs_lanes != 0 && cfg->rhs_lanes != 1 && cfg->rhs_lanes != 2 && cfg->rhs_lanes != 4 &&
        cfg->rhs_lanes != 8 && cfg->rhs_lanes != 16)
        return set_error(LQCD_EINVAL, "rhs_lanes %d not in {0, 1, 2, 4, 8, 16}", cfg->rhs_lanes);
    std::lock_guard<std::mutex> lk(g_launch_mu);
    g_launch[kernel][k] = Launch{cfg->block, cfg->swizzle, cfg->order, cfg->rhs_tile, cfg->rhs_group,
                                 cfg->ygroup < 1 ? 1 : cfg->ygroup, cfg->rhs_lanes < 1 ? 1 : cfg->rhs_lanes};
    return LQCD_OK;
}

int lqcd_get_launch(int32_t kernel, int32_t prec, lqcd_launch* cfg)
{
    if (kernel != LQCD_KERNEL_DSLASH && kernel != LQCD_KERNEL_BLAS && kernel != LQCD_KERNEL_STAG &&
        kernel != LQCD_KERNEL_DSLASH_RHS)
        return set_error(LQCD_EINVAL, "unknown kernel %d", kernel);
    const int k = prec_slot(prec);
    if (k < 0) return set_error(LQCD_EINVAL, "prec %d not in {64, 32, 16}", prec);
    if (!cfg) return set_error(LQCD_EINVAL, "cfg is NULL");
    const Launch l = launch_for(kernel, prec);
    cfg->block = l.block;
    cfg->swizzle = l.swizzle;
    cfg->order = l.order;
    cfg->rhs_tile = l.rhs_tile;
    cfg->rhs_group = l.rhs_group;
    cfg->ygroup = l.ygroup;
    cfg->rhs_lanes = l.rhs_lanes;
    return LQCD_OK;
}

namespace {
int tune_args(int32_t kernel, int32_t prec, int32_t recon, const lqcd_geom* geom, int32_t nrhs, Geom* g)
{
    if (kernel != LQCD_KERNEL_DSLASH && kernel != LQCD_KERNEL_STAG && kernel != LQCD_KERNEL_DSLASH_RHS)
        return set_error(LQCD_EINVAL, "kernel %d has no cached shapes (DSLASH, STAG or DSLASH_RHS)", kernel);
    if (prec_slot(prec) < 0) return set_error(LQCD_EINVAL, "prec %d not in {64, 32, 16}", prec);
    if (recon != 18 && recon != 12) return set_error(LQCD_EINVAL, "recon %d not 18 or 12", recon);
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(LQCD_EINVAL, "nrhs %d not in [1, %d]", nrhs, kMaxRhs);
    return make_geom(geom, g);
}
}  // namespace

int lqcd_tune_cache_load(const char* path)
{
    g_err[0] = 0;
    if (!path) return set_error(LQCD_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_init_locked();
    return tune_load_locked(path, false);
}

int lqcd_tune_cache_save(const char* path)
{
    g_err[0] = 0;
    if (!path) return set_error(LQCD_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_init_locked();
    return tune_save_locked(path);
}

int lqcd_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_env_read = true;  // an explicit clear also drops what the file would add
    g_tune.clear();
    return LQCD_OK;
}

int lqcd_tune_cache_put(int32_t kernel, int32_t prec, int32_t recon, const lqcd_geom* geom, int32_t nrhs,
                        const lqcd_launch* cfg, double us)
{
    g_err[0] = 0;
    Geom g;
    int rc = tune_args(kernel, prec, recon, geom, nrhs, &g);
    if (rc) return rc;
    if (!cfg) return set_error(LQCD_EINVAL, "cfg is NULL");
    const Launch l{cfg->block, cfg->swizzle, cfg->order, cfg->rhs_tile, cfg->rhs_group, cfg->ygroup, cfg->rhs_lanes};
    if (const char* bad = launch_problem(kernel, l)) return set_error(LQCD_EINVAL, "cfg: %s", bad);
    if (!std::isfinite(us) || us < 0) return set_error(LQCD_EINVAL, "us must be finite and >= 0");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_init_locked();
    g_tune[tune_key(kernel, prec, recon, g.L, nrhs)] = TuneVal{l, us};
    return LQCD_OK;
}

int lqcd_tune_cache_get(int32_t kernel, int32_t prec, int32_t recon, const lqcd_geom* geom, int32_t nrhs,
                        lqcd_launch* cfg, double* us, int32_t* found)
{
    g_err[0] = 0;
    Geom g;
    int rc = tune_args(kernel, prec, recon, geom, nrhs, &g);
    if (rc) return rc;
    if (!cfg || !found) return set_error(LQCD_EINVAL, "cfg or found is NULL");
    Launch l;
    bool hit = false;
    double t = 0.0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_env_init_locked();
        const auto it = g_tune.find(tune_key(kernel, prec, recon, g.L, nrhs));
        if (it != g_tune.end()) {
            hit = true;
            l = it->second.l;
            t = it->second.us;
        }
    }
    if (!hit) l = launch_for(kernel, prec);
    cfg->block = l.block;
    cfg->swizzle = l.swizzle;
    cfg->order = l.order;
    cfg->rhs_tile = l.rhs_tile;
    cfg->rhs_group = l.rhs_group;
    cfg->ygroup = l.ygroup;
    cfg->rhs_lanes = l.rhs_lanes;
    if (us) *us = t;
    *found = hit ? 1 : 0;
    return LQCD_OK;
}

int lqcd_autotune_dslash(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out,
                         int32_t reps, void* stream, lqcd_launch* best, double* best_us)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_op(op))) return rc;
    if (!U || !in || !out) return set_error(LQCD_EINVAL, "NULL field pointer");
    if (in == out) return set_error(LQCD_EINVAL, "in and out must not alias");
    if (reps < 1 || reps > 10000) return set_error(LQCD_EINVAL, "reps %d out of range", reps);
    Op o;
    o.g = g;
    o.prec = op->prec;
    o.recon = op->recon;
    o.U = U;
    o.kappa = op->kappa;
    o.mu = op->mu;
    o.nrhs = 1;
    o.pb = parity_bytes(g, op->prec);
    o.s = static_cast<hipStream_t>(stream);
    return autotune_hop(LQCD_KERNEL_DSLASH, op->prec, op->recon, g.L, reps, o.s, best, best_us, [&](const Launch& cfg) {
        o.dcfg = cfg;
        return o.hop(0, in, out, false, SpinCoef{}, nullptr, coef_real(1.0), nullptr, RED_NONE, FIN_STORE,
                     PRED_ALWAYS);
    });
}

int lqcd_autotune_dslash_rhs(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out,
                             int32_t nrhs, int32_t reps, void* stream, lqcd_launch* best, double* best_us)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_op(op))) return rc;
    if (!U || !in || !out) return set_error(LQCD_EINVAL, "NULL field pointer");
    if (in == out) return set_error(LQCD_EINVAL, "in and out must not alias");
    if (nrhs < 2 || nrhs > kMaxRhs) return set_error(LQCD_EINVAL, "nrhs %d not in [2, %d]", nrhs, kMaxRhs);
    if (reps < 1 || reps > 10000) return set_error(LQCD_EINVAL, "reps %d out of range", reps);
    Op o;
    o.g = g;
    o.prec = op->prec;
    o.recon = op->recon;
    o.U = U;
    o.kappa = op->kappa;
    o.mu = op->mu;
    o.nrhs = nrhs;
    o.pb = parity_bytes(g, op->prec);
    o.s = static_cast<hipStream_t>(stream);
    const Launch shape = launch_for(LQCD_KERNEL_DSLASH_RHS, op->prec);
    hipEvent_t e0, e1;
    LQCD_HIP(hipEventCreate(&e0));
    LQCD_HIP(hipEventCreate(&e1));
    Launch win = shape;
    float win_ms = 0.f;
    bool have = false;
    int result = LQCD_OK;
    const int blocks[3] = {128, 192, 256};
    const int tiles[3] = {1, 2, 4};
    const int groups[5] = {0, 2, 4, 8, 16};
    const int lanes[4] = {2, 4, 8, 16};
    for (int bi = 0; bi < 3 && !result; ++bi) {
        // tiles 1, 2, 4 in registers with groups, then tile 1 across 2..16 lanes
        for (int ti = 0; ti < 3 + 4 && !result; ++ti) {
            const bool across = ti >= 3;
            const int tile = across ? 1 : tiles[ti];
            if (!across && dslash_rhs_tile(op->prec, tile, nrhs) != tile) continue;  // not compiled / larger than nrhs
            if (across && (shape.order < 1 || lanes[ti - 3] > 2 * nrhs)) continue;
            for (int gi = 0; gi < (across ? 1 : 5) && !result; ++gi) {
                Launch cfg = shape;
                cfg.block = blocks[bi];
                cfg.rhs_tile = tile;
                cfg.rhs_group = across ? 0 : groups[gi];
                cfg.rhs_lanes = across ? lanes[ti - 3] : 1;
                o.dcfg = cfg;
                auto hop = [&]() {
                    return o.hop(0, in, out, false, SpinCoef{}, nullptr, coef_real(1.0), nullptr, RED_NONE, FIN_STORE,
                                 PRED_ALWAYS);
                };
                hipError_t e = hipSuccess;
                for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hop();
                if (e == hipSuccess) e = hipEventRecord(e0, o.s);
                for (int i = 0; i < reps && e == hipSuccess; ++i) e = hop();
                if (e == hipSuccess) e = hipEventRecord(e1, o.s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    result = set_error(LQCD_EHIP, "autotune: %s", hipGetErrorString(e));
                    break;
                }
                if (!have || ms < win_ms) {
                    have = true;
                    win_ms = ms;
                    win = cfg;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result) return result;
    {
        std::lock_guard<std::mutex> lk(g_launch_mu);
        g_launch[LQCD_KERNEL_DSLASH_RHS][prec_slot(op->prec)] = win;
    }
    tune_record(LQCD_KERNEL_DSLASH_RHS, op->prec, op->recon, g.L, nrhs, win, 1e3 * win_ms / reps);
    if (best) {
        best->block = win.block;
        best->swizzle = win.swizzle;
        best->order = win.order;
        best->rhs_tile = win.rhs_tile;
        best->rhs_group = win.rhs_group;
        best->ygroup = win.ygroup;
        best->rhs_lanes = win.rhs_lanes;
    }
    if (best_us) *best_us = 1e3 * win_ms / reps;
    return LQCD_OK;
}

int lqcd_autotune_stag(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* in, void* out,
                       int32_t reps, void* stream, lqcd_launch* best, double* best_us)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_stag_op(op))) return rc;
    if (!U || !in || !out) return set_error(LQCD_EINVAL, "NULL field pointer");
    if (in == out) return set_error(LQCD_EINVAL, "in and out must not alias");
    if (reps < 1 || reps > 10000) return set_error(LQCD_EINVAL, "reps %d out of range", reps);
    StagOp o;
    o.g = g;
    o.prec = op->prec;
    o.recon = op->recon;
    o.U = U;
    o.mass = op->mass;
    o.nrhs = 1;
    o.pb = colour_bytes(g, op->prec);
    o.s = static_cast<hipStream_t>(stream);
    return autotune_hop(LQCD_KERNEL_STAG, op->prec, op->recon, g.L, reps, o.s, best, best_us, [&](const Launch& cfg) {
        o.dcfg = cfg;
        return o.hop(0, in, out, 0.5, nullptr, 0.0, nullptr, RED_NONE, FIN_STORE, PRED_ALWAYS, nullptr);
    });
}

int lqcd_pack_gauge(const lqcd_geom* geom, int32_t prec, int32_t recon, const void* U_canonical, void* U_out,
                    void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_prec(prec, recon))) return rc;
    if (!U_canonical || !U_out) return set_error(LQCD_EINVAL, "NULL pointer");
    LQCD_K(launch_pack_gauge(prec, recon, g, U_canonical, U_out, static_cast<hipStream_t>(stream)));
    return LQCD_OK;
}

int lqcd_pack_spinor(const lqcd_geom* geom, int32_t prec, int32_t nrhs, const void* psi, void* out, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_prec(prec, 12))) return rc;
    if (nrhs < 1 || nrhs > 65535) return set_error(LQCD_EINVAL, "nrhs %d out of range", nrhs);
    if (!psi || !out) return set_error(LQCD_EINVAL, "NULL pointer");
    LQCD_K(launch_pack_spinor(prec, g, psi, out, nrhs, static_cast<hipStream_t>(stream)));
    return LQCD_OK;
}

int lqcd_unpack_spinor(const lqcd_geom* geom, int32_t prec, int32_t nrhs, const void* in, void* psi, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_prec(prec, 12))) return rc;
    if (nrhs < 1 || nrhs > 65535) return set_error(LQCD_EINVAL, "nrhs %d out of range", nrhs);
    if (!psi || !in) return set_error(LQCD_EINVAL, "NULL pointer");
    LQCD_K(launch_unpack_spinor(prec, g, in, psi, nrhs, static_cast<hipStream_t>(stream)));
    return LQCD_OK;
}

int dslash_apply(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out, int32_t dagger,
                 int32_t nrhs, void* ws, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_op(op))) return rc;
    if (!U || !in || !out) return set_error(LQCD_EINVAL, "NULL field pointer");
    if (in == out) return set_error(LQCD_EINVAL, "in and out must not alias");
    if (nrhs < 1 || nrhs > 65535) return set_error(LQCD_EINVAL, "nrhs %d out of range", nrhs);
    (void)ws;
    Op o;
    o.g = g;
    o.prec = op->prec;
    o.recon = op->recon;
    o.U = U;
    o.kappa = op->kappa;
    o.mu = op->mu;
    o.nrhs = nrhs;
    o.pb = parity_bytes(g, op->prec);
    o.s = static_cast<hipStream_t>(stream);
    o.tune();
    LQCD_K(o.full_M(in, out, dagger != 0, 1.0, nullptr, RED_NONE, FIN_STORE, PRED_ALWAYS));
    return LQCD_OK;
}

int dslash_eo_apply(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out,
                    int32_t out_parity, int32_t op_kind, int32_t dagger, int32_t nrhs, void* ws, void* stream)
{
    Geom g;
    int rc = eo_apply_check(geom, op, U, in, out, out_parity, op_kind, nrhs, &g);
    if (rc) return rc;
    void* tmp = nullptr;
    if (op_kind == LQCD_OP_SCHUR) {
        if (!ws) return set_error(LQCD_EINVAL, "LQCD_OP_SCHUR needs a workspace");
        Arena ar{static_cast<char*>(ws), 0, 0};
        RedScratch rs;
        plan_reductions(ar, g, kMaxRhs, &rs);
        tmp = ar.take((size_t)(parity_bytes(g, op->prec) * nrhs));
    }
    return eo_apply_run(g, op, U, in, out, out_parity, op_kind, dagger, nrhs, tmp, stream);
}

int dslash_eo_apply_noalloc(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out,
                            int32_t out_parity, int32_t op_kind, int32_t dagger, int32_t nrhs, void* stream)
{
    Geom g;
    int rc = eo_apply_check(geom, op, U, in, out, out_parity, op_kind, nrhs, &g);
    if (rc) return rc;
    void* tmp = nullptr;
    if (op_kind == LQCD_OP_SCHUR) {
        const size_t need = (size_t)(parity_bytes(g, op->prec) * nrhs);
        if (need > kScratchBytes)
            return set_error(LQCD_EINVAL,
                             "dslash_eo_apply_noalloc: the odd-parity temporary needs %zu bytes, more than the "
                             "library's %zu-byte device array (use dslash_eo_apply with a workspace)",
                             need, kScratchBytes);
        if ((rc = scratch_address(&tmp))) return rc;
    }
    return eo_apply_run(g, op, U, in, out, out_parity, op_kind, dagger, nrhs, tmp, stream);
}

int cg_solve(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* b, void* x,
             const lqcd_solve_params* params, lqcd_solve_info* info, void* ws, size_t ws_bytes, void* stream)
{
    return solve(M_CG, geom, op, U, b, x, params, info, ws, ws_bytes, stream);
}

int bicgstab_solve(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* b, void* x,
                   const lqcd_solve_params* params, lqcd_solve_info* info, void* ws, size_t ws_bytes,
                   void* stream)
{
    return solve(M_BICG, geom, op, U, b, x, params, info, ws, ws_bytes, stream);
}

int lqcd_workspace_bytes_batch(int32_t nsys, const lqcd_geom* geoms, const lqcd_op* ops,
                               const lqcd_solve_params* params, size_t* bytes)
{
    if (nsys < 1 || nsys > kMaxSys) return set_error(LQCD_EINVAL, "nsys %d not in [1, %d]", nsys, kMaxSys);
    if (!geoms || !ops || !bytes) return set_error(LQCD_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_params(params, M_CG))) return rc;
    std::vector<Geom> g(nsys);
    for (int s = 0; s < nsys; ++s) {
        if ((rc = make_geom(&geoms[s], &g[s]))) return rc;
        if ((rc = check_op(&ops[s]))) return rc;
    }
    BatchLayout L;
    plan_batch(nsys, g.data(), ops, params, nullptr, &L);
    *bytes = L.bytes;
    return LQCD_OK;
}

int cg_solve_batch(int32_t nsys, const lqcd_geom* geoms, const lqcd_op* ops, const void* const* U,
                   const void* const* b, void* const* x, const lqcd_solve_params* params, lqcd_solve_info* info,
                   void* ws, size_t ws_bytes, void* stream)
{
    return solve_batch(nsys, geoms, ops, U, b, x, params, info, ws, ws_bytes, stream);
}

int lqcd_autotune_batch(int32_t nsys, const lqcd_geom* geoms, const lqcd_op* ops, const void* const* U,
                        const void* const* b, void* const* x, const lqcd_solve_params* params, void* ws,
                        size_t ws_bytes, int32_t iters, void* stream, lqcd_launch* best, double* best_us)
{
    return autotune_batch(nsys, geoms, ops, U, b, x, params, ws, ws_bytes, iters, stream, best, best_us);
}


// ---------------------------------------------------------------------------
// Staggered fermions

int lqcd_pack_colour(const lqcd_geom* geom, int32_t prec, int32_t nrhs, const void* chi, void* out, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_prec(prec, 12))) return rc;
    if (nrhs < 1 || nrhs > 65535) return set_error(LQCD_EINVAL, "nrhs %d out of range", nrhs);
    if (!chi || !out) return set_error(LQCD_EINVAL, "NULL pointer");
    LQCD_K(launch_pack_colour(prec, g, chi, out, nrhs, static_cast<hipStream_t>(stream)));
    return LQCD_OK;
}

int lqcd_unpack_colour(const lqcd_geom* geom, int32_t prec, int32_t nrhs, const void* in, void* chi, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_prec(prec, 12))) return rc;
    if (nrhs < 1 || nrhs > 65535) return set_error(LQCD_EINVAL, "nrhs %d out of range", nrhs);
    if (!chi || !in) return set_error(LQCD_EINVAL, "NULL pointer");
    LQCD_K(launch_unpack_colour(prec, g, in, chi, nrhs, static_cast<hipStream_t>(stream)));
    return LQCD_OK;
}

int stag_apply(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* in, void* out, int32_t dagger,
               int32_t nrhs, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_stag_op(op))) return rc;
    if (!U || !in || !out) return set_error(LQCD_EINVAL, "NULL field pointer");
    if (in == out) return set_error(LQCD_EINVAL, "in and out must not alias");
    if (nrhs < 1 || nrhs > 65535) return set_error(LQCD_EINVAL, "nrhs %d out of range", nrhs);
    StagOp o;
    o.g = g;
    o.prec = op->prec;
    o.recon = op->recon;
    o.U = U;
    o.mass = op->mass;
    o.nrhs = nrhs;
    o.pb = colour_bytes(g, op->prec);
    o.s = static_cast<hipStream_t>(stream);
    o.tune();
    LQCD_K(o.full_M(in, out, dagger != 0, 1.0, nullptr, RED_NONE, FIN_STORE, PRED_ALWAYS, nullptr));
    return LQCD_OK;
}

int stag_eo_apply(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* in, void* out,
                  int32_t out_parity, int32_t op_kind, int32_t nrhs, void* ws, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_stag_op(op))) return rc;
    if (!U || !in || !out) return set_error(LQCD_EINVAL, "NULL field pointer");
    if (in == out) return set_error(LQCD_EINVAL, "in and out must not alias");
    if (out_parity != 0 && out_parity != 1) return set_error(LQCD_EINVAL, "out_parity must be 0 or 1");
    if (nrhs < 1 || nrhs > 65535) return set_error(LQCD_EINVAL, "nrhs %d out of range", nrhs);
    StagOp o;
    o.g = g;
    o.prec = op->prec;
    o.recon = op->recon;
    o.U = U;
    o.mass = op->mass;
    o.nrhs = nrhs;
    o.pb = colour_bytes(g, op->prec);
    o.s = static_cast<hipStream_t>(stream);
    o.tune();
    if (op_kind == LQCD_OP_HOP) {
        LQCD_K(o.hop(out_parity, in, out, 0.5, nullptr, 0.0, nullptr, RED_NONE, FIN_STORE, PRED_ALWAYS, nullptr));
        return LQCD_OK;
    }
    if (op_kind == LQCD_OP_NORMAL) {
        if (out_parity != 0) return set_error(LQCD_EINVAL, "the normal operator acts on even sites (out_parity 0)");
        if (!ws) return set_error(LQCD_EINVAL, "LQCD_OP_NORMAL needs a workspace of nrhs odd fields");
        LQCD_K(o.normal(in, out, ws, 0.0, 1.0, nullptr, RED_NONE, FIN_STORE, PRED_ALWAYS, nullptr));
        return LQCD_OK;
    }
    return set_error(LQCD_EINVAL, "unknown op_kind %d for staggered fermions", op_kind);
}

int lqcd_workspace_bytes_stag(const lqcd_geom* geom, const lqcd_stag_op* op, int32_t nshift, size_t* bytes)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_stag_op(op))) return rc;
    if (!bytes) return set_error(LQCD_EINVAL, "bytes is NULL");
    if (nshift < 0 || nshift > kMaxShifts) return set_error(LQCD_EINVAL, "nshift %d not in [0, %d]", nshift, kMaxShifts);
    StagPlan sp;
    plan_stag(g, nshift, nullptr, &sp);
    *bytes = sp.bytes;
    return LQCD_OK;
}

int stag_cg_solve(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* b, void* x,
                  const lqcd_solve_params* prm, lqcd_solve_info* info, void* ws, size_t ws_bytes, void* stream)
{
    const double t0 = now_s();
    g_err[0] = 0;
    Geom g;
    int rc = stag_validate(geom, op, U, b, x, prm, info, ws, stream, &g);
    if (rc) return rc;
    StagPlan sp;
    plan_stag(g, 0, ws, &sp);
    if (ws_bytes < sp.bytes) return set_error(LQCD_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, sp.bytes);
    const StagOp o = stag_bind(g, op, U, sp, stream);
    const int64_t pb = o.pb;
    const char* bc = static_cast<const char*>(b);
    char* xc = static_cast<char*>(x);
    Ctl* ctl = sp.rs.ctl;
    const double m = op->mass;

    // stop on ||r_e|| <= tol m ||b||: tol2 = (tol m)^2, bb = ||b||^2 (full)
    LQCD_K(launch_ctl_init(ctl, 1, prm->tol * m, 0.0, prm->maxiter, o.s));
    ShiftList sl{};
    LQCD_K(launch_ctl_init_shifts(ctl, 1, 0, sl, o.s));
    LQCD_K(o.blas(BLAS_NORM, 1, PRED_ALWAYS, FIN_BB_FULL, ctl, const_cast<char*>(bc), 2 * pb, nullptr, 0, nullptr, 0,
                  nullptr, 0, 2));
    // bhat = m b_e - D_eo b_o ; x_e = 0
    LQCD_K(o.hop(0, bc + pb, sp.bhat, -0.5, bc, m, nullptr, RED_NONE, FIN_STORE, PRED_ALWAYS, ctl));
    LQCD_K(o.blas(BLAS_ZERO, 1, PRED_ALWAYS, FIN_STORE, ctl, nullptr, 0, xc, 2 * pb));

    int restarts = 0;
    for (int pass = 0;; ++pass) {
        // r = bhat - N x_e (bhat itself on the first pass) ; p = r ; rr
        if (pass == 0) LQCD_K(o.blas(BLAS_COPY, 1, PRED_ACTIVE, FIN_STORE, ctl, sp.bhat, pb, sp.r, pb));
        else LQCD_K(o.normal(xc, sp.r, sp.t, 0.0, -1.0, sp.bhat, RED_NONE, FIN_STORE, PRED_ACTIVE, ctl));
        LQCD_K(o.blas(BLAS_COPY, 1, PRED_ACTIVE, FIN_STORE, ctl, sp.r, pb, sp.p, pb));
        LQCD_K(o.blas(BLAS_NORM, 1, PRED_ACTIVE, FIN_MS_INIT_KEEP, ctl, sp.r, pb));
        const int chunk = prm->check_every > 0 ? prm->check_every : 8;
        rc = drive(o.s, ctl, 1, 1, 1, chunk, prm->maxiter, prm->use_graph != 0,
                   [&]() { return stag_ms_iter(o, sp, xc, 1, 0, 0.0); });
        if (rc) return rc;
        // x_o = (b_o - D_oe x_e) / m ; true residual ||b - M x||^2
        LQCD_K(o.hop(1, xc, xc + pb, -0.5 / m, bc + pb, 1.0 / m, nullptr, RED_NONE, FIN_STORE, PRED_ALWAYS, ctl));
        LQCD_K(o.full_M(xc, nullptr, false, -1.0, bc, RED_NORM, FIN_TRUE_RR, PRED_ALWAYS, ctl));
        std::vector<Ctl> h;
        if ((rc = read_ctls(o.s, ctl, 1, h))) return rc;
        const double tr = h[0].bb > 0 ? std::sqrt(h[0].true_rr / h[0].bb) : 0.0;
        if (h[0].status != 0 || tr <= prm->tol || h[0].iter >= prm->maxiter || restarts >= 8) break;
        ++restarts;
        LQCD_K(launch_ctl_reopen(ctl, 1, 1u, o.s));
    }
    std::vector<Ctl> h;
    if ((rc = read_ctls(o.s, ctl, 1, h))) return rc;
    lqcd_solve_info& in = info[0];
    in.iters = h[0].iter;
    in.reliable_updates = 0;
    in.restarts = restarts;
    in.true_resid = h[0].bb > 0 ? std::sqrt(h[0].true_rr / h[0].bb) : 0.0;
    in.eo_resid = std::nan("");
    in.seconds = now_s() - t0;
    // even-odd hops: bhat 1, 2 per iteration and per restart residual, reconstruct 1 and full M 2 per pass
    in.hops_outer = 1.0 + 2.0 * h[0].iter + 2.0 * restarts + 3.0 * (restarts + 1);
    in.hops_inner = 0.0;
    int st = h[0].status;
    if (st == LQCD_OK && in.true_resid > prm->tol) st = LQCD_ENOCONV;
    if (st == LQCD_OK && !std::isfinite(in.true_resid)) st = LQCD_ENONFINITE;
    in.status = st;
    return st;
}

int stag_multishift_solve(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* b, void* x,
                          const double* shifts, int32_t nshift, const lqcd_solve_params* prm, lqcd_solve_info* info,
                          void* ws, size_t ws_bytes, void* stream)
{
    const double t0 = now_s();
    g_err[0] = 0;
    Geom g;
    int rc = stag_validate(geom, op, U, b, x, prm, info, ws, stream, &g);
    if (rc) return rc;
    if (!shifts) return set_error(LQCD_EINVAL, "shifts is NULL");
    if (nshift < 1 || nshift > kMaxShifts) return set_error(LQCD_EINVAL, "nshift %d not in [1, %d]", nshift, kMaxShifts);
    ShiftList sl{};
    int base = 0;
    for (int i = 0; i < nshift; ++i) {
        if (!std::isfinite(shifts[i]) || shifts[i] < 0.0) return set_error(LQCD_EINVAL, "shift %d must be finite and >= 0", i);
        sl.s[i] = shifts[i];
        if (shifts[i] < shifts[base]) base = i;
    }
    StagPlan sp;
    plan_stag(g, nshift, ws, &sp);
    if (ws_bytes < sp.bytes) return set_error(LQCD_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, sp.bytes);
    const StagOp o = stag_bind(g, op, U, sp, stream);
    const int64_t pb = o.pb;
    char* bc = static_cast<char*>(const_cast<void*>(b));
    char* xc = static_cast<char*>(x);
    Ctl* ctl = sp.rs.ctl;

    // x_i = 0 ; r = b ; p_i = b ; ||b||^2 sets every shift's threshold
    LQCD_K(launch_ctl_init(ctl, nshift, prm->tol, 0.0, prm->maxiter, o.s));
    LQCD_K(launch_ctl_init_shifts(ctl, nshift, base, sl, o.s));
    LQCD_K(o.blas(BLAS_ZERO, nshift, PRED_ALWAYS, FIN_STORE, ctl, nullptr, 0, xc, pb));
    LQCD_K(o.blas(BLAS_COPY, 1, PRED_ALWAYS, FIN_STORE, ctl, bc, pb, sp.r, pb));
    LQCD_K(o.blas(BLAS_COPY, nshift, PRED_ALWAYS, FIN_STORE, ctl, bc, 0, sp.p, pb));
    LQCD_K(o.blas(BLAS_NORM, 1, PRED_ALWAYS, FIN_MS_INIT, ctl + base, bc, pb));
    const int chunk = prm->check_every > 0 ? prm->check_every : 8;
    rc = drive(o.s, ctl, 1, nshift, nshift, chunk, prm->maxiter, prm->use_graph != 0,
               [&]() { return stag_ms_iter(o, sp, xc, nshift, base, sl.s[base]); });
    if (rc) return rc;
    // true residuals ||b - (N + s_i) x_i||^2, one system at a time
    for (int i = 0; i < nshift; ++i)
        LQCD_K(o.normal(xc + i * pb, nullptr, sp.t, sl.s[i], -1.0, bc, RED_NORM, FIN_TRUE_RR, PRED_ALWAYS, ctl + i));
    std::vector<Ctl> h;
    if ((rc = read_ctls(o.s, ctl, nshift, h))) return rc;
    const int ms_iters = h[base].iter;
    std::vector<int> iters(nshift), ms_own(nshift), passes(nshift, 0);
    for (int i = 0; i < nshift; ++i) iters[i] = ms_own[i] = h[i].iter;
    auto true_res = [&](const Ctl& c) { return c.bb > 0 ? std::sqrt(c.true_rr / c.bb) : 0.0; };

    // Every shift must meet tol by its FP64 true residual.  A shift whose
    // recursion stopped on |zeta| ||r|| but whose recomputed residual misses
    // (rounding of the shifted recurrences) is refined by a single-shift CG on
    // (N + s_i) started from its x_i; p_i, no longer needed by the family,
    // serves as its search direction.
    for (int pass = 0; pass < kMaxRefine; ++pass) {
        bool any = false;
        for (int i = 0; i < nshift; ++i) {
            if (h[i].status != LQCD_OK || true_res(h[i]) <= prm->tol || iters[i] >= prm->maxiter) continue;
            any = true;
            ++passes[i];
            Ctl* ci = ctl + i;
            StagPlan si = sp;
            si.rs.ctl = ci;
            si.p = static_cast<char*>(sp.p) + i * pb;
            char* xi = xc + i * pb;
            CtlInit in{};
            in.tol = prm->tol;
            in.iter_limit = prm->maxiter - iters[i];
            ShiftList one{};
            LQCD_K(launch_ctl_init(ci, 1, in, o.s));
            LQCD_K(launch_ctl_init_shifts(ci, 1, 0, one, o.s));
            LQCD_K(o.blas(BLAS_NORM, 1, PRED_ALWAYS, FIN_BB_FULL, ci, bc, pb));
            // r = b - (N + s_i) x_i ; p = r ; rr
            LQCD_K(o.normal(xi, sp.r, sp.t, sl.s[i], -1.0, bc, RED_NONE, FIN_STORE, PRED_ACTIVE, ci));
            LQCD_K(o.blas(BLAS_COPY, 1, PRED_ACTIVE, FIN_STORE, ci, sp.r, pb, si.p, pb));
            LQCD_K(o.blas(BLAS_NORM, 1, PRED_ACTIVE, FIN_MS_INIT_KEEP, ci, sp.r, pb));
            const int chunk = prm->check_every > 0 ? prm->check_every : 8;
            rc = drive(o.s, ci, 1, 1, 1, chunk, in.iter_limit, prm->use_graph != 0,
                       [&]() { return stag_ms_iter(o, si, xi, 1, 0, sl.s[i]); });
            if (rc) return rc;
            LQCD_K(o.normal(xi, nullptr, sp.t, sl.s[i], -1.0, bc, RED_NORM, FIN_TRUE_RR, PRED_ALWAYS, ci));
            std::vector<Ctl> hi;
            if ((rc = read_ctls(o.s, ci, 1, hi))) return rc;
            iters[i] += hi[0].iter;
            h[i] = hi[0];
        }
        if (!any) break;
    }

    const double secs = now_s() - t0;
    int worst = LQCD_OK;
    for (int i = 0; i < nshift; ++i) {
        lqcd_solve_info& in = info[i];
        in = lqcd_solve_info{};
        in.iters = iters[i];
        in.reliable_updates = 0;
        in.restarts = passes[i];
        in.true_resid = true_res(h[i]);
        in.eo_resid = std::nan("");
        in.seconds = secs;
        // the shared iterations are counted on every system: 2 hops each, plus
        // its true residual; a refinement adds its own iterations, residual
        // and true residual
        in.hops_outer = 2.0 * ms_iters + 2.0 + 2.0 * (iters[i] - ms_own[i]) + 4.0 * passes[i];
        in.hops_inner = 0.0;
        in.outer_iters = 1;
        int st = h[i].status;
        if (st == LQCD_OK && !(in.true_resid <= prm->tol)) st = LQCD_ENOCONV;
        in.status = st;
        if (st != LQCD_OK && worst == LQCD_OK) worst = st;
    }
    return worst;
}

// ---------------------------------------------------------------------------
// Twisted-mass pseudo-fermion force (the HMC's fermion part)

int lqcd_gamma5(const lqcd_geom* geom, int32_t nrhs, const void* in, void* out, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if (!in || !out) return set_error(LQCD_EINVAL, "NULL field pointer");
    if (nrhs < 1 || nrhs > 65535) return set_error(LQCD_EINVAL, "nrhs %d out of range", nrhs);
    BlasArgs a{};
    a.kind = KIND_SPINOR;
    a.Vh = g.Vh;
    a.S = g.S;
    a.nsub = 2;
    a.sub_stride = parity_bytes(g, 64);
    a.pred = PRED_ALWAYS;
    a.x = const_cast<void*>(in);
    a.y = out;
    a.st_x = a.st_y = 2 * parity_bytes(g, 64);
    a.coef = SpinCoef{{1.0, 0.0}, {-1.0, 0.0}};
    a.r.fin = FIN_STORE;
    LQCD_K(launch_blas(64, BLAS_SPIN_SCALE, a, nrhs, launch_for(LQCD_KERNEL_BLAS, 64), static_cast<hipStream_t>(stream)));
    return LQCD_OK;
}

int tm_force(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* X, const void* Wf, void* F,
             double scale, int32_t accumulate, void* stream)
{
    Geom g;
    int rc = make_geom(geom, &g);
    if (rc) return rc;
    if ((rc = check_op(op))) return rc;
    if (op->prec != 64) return set_error(LQCD_EINVAL, "the force takes FP64 fields (op->prec = 64)");
    if (!U || !X || !Wf || !F) return set_error(LQCD_EINVAL, "NULL pointer");
    if (accumulate != 0 && accumulate != 1) return set_error(LQCD_EINVAL, "accumulate must be 0 or 1");
    if (!std::isfinite(scale)) return set_error(LQCD_EINVAL, "scale must be finite");
    if (384 * g.S > INT32_MAX || 2 * (int64_t)g.Vh * 144 > INT32_MAX)
        return set_error(LQCD_EINVAL, "lattice too large for the force kernel: a full-lattice FP64 spinor field "
                                      "and one direction of F must each stay under 2 GiB (about 11 million sites)");
    LQCD_K(launch_tm_force(op->recon, g, U, X, Wf, F, op->kappa, scale, accumulate, static_cast<hipStream_t>(stream)));
    return LQCD_OK;
}
}  // extern "C"
