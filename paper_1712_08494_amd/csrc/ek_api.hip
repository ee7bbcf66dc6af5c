// Host runtime of the coupled electrokinetic lattice library: context set-up (geometry,
// device memory, initial state), the step loop, the Poisson convergence control and the
// export calls of include/ek.h.  All per-step arithmetic runs in the kernels of
// ek_kernels.hip; the host only orders launches and reads back scalars.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <hipfft/hipfft.h>

#include "ek.h"
#include "ek_device.h"
#include "ek_internal.h"
#include "ek_lattice.h"

using namespace ek;

namespace ek {
template <typename T>
void launch_init_pop_flags(const Scalars& S, T* f, const double* rho, double rref, const uint8_t* flags, hipStream_t st);
}

struct TimeRec {
    hipEvent_t a, b;
    int cls;
    int count;
};

struct ek_ctx {
    ek_params p{};
    // device memory: hipMalloc (ws_mode 0), or carved from the caller's workspace (2); 1 only
    // adds up the sizes (ek_workspace_bytes)
    char* ws = nullptr;
    size_t ws_size = 0, ws_used = 0;
    int ws_mode = 0;
    bool split_layout = false;  // multigrid solves on colour-split copies of potential and charge
    bool one_pass = false;      // lattice sweeps of a colour-split solve in one pass (k_sor_rb) where it fits
    int fixed_cycles = 0;       // > 0: that many V-cycles per step, no host read-back (ek_params.poisson_cycles)
    double rel_max = 0.0;       // largest relative residual of the solves since the last ek_observables
    double* obs_scratch = nullptr;  // this device's address of the library's observables scratch array
    hipStream_t st = nullptr;
    std::string err;
    Scalars S{};
    unsigned N = 0, nblk = 0;
    size_t esz = 8;
    std::vector<void*> allocs;
    size_t bytes = 0;
    // fields
    void* f[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [buffer][component]
    void* n[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [buffer][species]
    void* mom = nullptr;
    void* uph = nullptr;
    void* q = nullptr;
    void* eps = nullptr;
    double* phi = nullptr;
    double* phi_prev = nullptr;  // potential of the previous step (time extrapolation)
    double* phi_prev2 = nullptr; // potential two steps back
    int phi_history = 0;         // potentials the warm start extrapolates from (1, 2 or 3; 0 adaptive)
    // adaptive warm start: the last start residual measured with linear (2) and quadratic
    // (3) extrapolation, the order in use and the steps since the other one was probed
    double rel0_of[4] = {0, 0, 0, 0};
    int ws_order = 2, ws_since = 0;
    int cur = 0;
    // geometry
    uint8_t* flags = nullptr;
    void* psif = nullptr;
    void* qc = nullptr;
    int32_t* owner = nullptr;
    int32_t* linkbase = nullptr;
    double* linkdp = nullptr;
    int32_t* vlist = nullptr;
    int nv = 0;
    int32_t* plist = nullptr;  // sites of the particle path
    int npl = 0;               // their number; with moving particles the list's capacity
    int32_t* npl_dev = nullptr;  // moving particles: the list's length, rebuilt on the device every step
    long long nlinks = 0;
    std::vector<uint8_t> hflags;   // host copy (solid marks for export)
    std::vector<double> hpsis;     // host copy of the solid fraction
    // particles
    int np = 0;
    double* px[2] = {nullptr, nullptr};
    double* pv[2] = {nullptr, nullptr};
    double* prad = nullptr;
    double* pF = nullptr;
    int pcur = 0;
    int32_t *plink_off = nullptr, *plink_idx = nullptr, *psite_off = nullptr, *psite_idx = nullptr;
    // moving particles projected anew (ek_params.reproject): particle charges, the geometry
    // copies and the work arrays of the projection (Reproj)
    double* pQ = nullptr;
    uint8_t* flags_old = nullptr;
    int32_t* owner_old = nullptr;
    void* psif_old = nullptr;
    int32_t* rp_origin = nullptr;
    int32_t *rp_nb = nullptr, *rp_nnb = nullptr;  // particles whose projection boxes meet
    int16_t* rp_cnt = nullptr;
    uint8_t *rp_inside = nullptr, *rp_event = nullptr;
    double *rp_evm = nullptr, *rp_ptot = nullptr;
    void* rp_share = nullptr;
    std::vector<double> px0, hrad;
    // scratch
    double* red = nullptr;
    double* scal = nullptr;
    double* hscal = nullptr;  // pinned
    int* obs_max = nullptr;
    double* stage = nullptr;
    double* stage2 = nullptr;
    // bookkeeping
    long long steps = 0, ptotal = 0;
    int last_iters = 0;
    double last_rel = 0.0, last_mean = 0.0, last_rel0 = 0.0;
    double omega = 1.0;
    double rate = -1.0;
    // multigrid (levels[0] is the lattice itself and holds no arrays)
    std::vector<MGLevel> mg;
    double mg_coarse_omega = 1.0;
    // V-cycle shape: red-black sweeps before and after the coarse correction on the
    // lattice and on the coarse grids, and sweeps on the coarsest grid
    int mg_fine_pre = 1, mg_fine_post = 2, mg_pre = 1, mg_post = 2, mg_coarsest = 10;
    int mg_tail_pre = 3, mg_tail_post = 3;  // sweeps on the upper grid of the single-workgroup tail
    double mg_omega = 1.2;  // relaxation of the smoothing sweeps (1: Gauss-Seidel)
    // One V-cycle captured as a HIP graph and replayed for each cycle of a solve (one host
    // call instead of ~40 launches).  It is captured with the context's own charge and
    // potential buffers (or their colour-split copies) and used only while they are the ones
    // in place; per-sweep timing (level 2) and a changed cycle shape fall back to direct
    // launches / a new capture.
    hipStream_t cap_st = nullptr;
    hipGraph_t vc_graph = nullptr;
    hipGraphExec_t vc_exec = nullptr;
    void* q_own = nullptr;
    double* phis = nullptr;  // colour-split potential and charge of a multigrid solve
    void* qs = nullptr;
    double* blk = nullptr;   // black values between the fused interpolation + red pass and the black pass
    double* phi_own = nullptr;
    // Set by the reverse sweep around its adjoint solve: the adjoint potential and its
    // source stand in for phi and q, and the solve runs like one of the own potential
    // (colour-split copies, the captured cycle, the cycle-count floor of its own history).
    bool adj_solve = false;
    bool vc_off = false;
    bool vc_split = false;  // layout the captured V-cycle graph works on
    int kring[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // V-cycles of the last own multigrid solves
    int kpos = 0;
    int kcount = 0;  // entries of kring recorded (at most 8)
    void* tune_buf = nullptr;  // state copy of the autotuner (held only while it runs)
    // tau = 1 moment state instead of populations (ek_params.moment_state): two buffers of
    // 8 N values (step parity as the populations), the FP64 initial densities the first
    // moments pass reads, and whether a step has written a moment state yet
    bool moment_state = false;
    // the lagged Fourier Poisson scheme (EK_POISSON_FFT): plans on the context's stream,
    // the right-hand side (N doubles) and the spectrum (nz ny (nx/2+1) complex doubles)
    bool fft = false;
    hipfftHandle fft_fwd = 0, fft_inv = 0;
    double* fft_rhs = nullptr;
    double* fft_spec = nullptr;
    double* fft_tab = nullptr;  // per-axis eigenvalue parts (nx/2 + 1 + ny + nz doubles)
    void* ms[2] = {nullptr, nullptr};
    double* rho0 = nullptr;
    // FP32 exact-mass collision (see Fields::rlo, Fields::mlo): 2 N floats each
    void* rlo = nullptr;
    void* mlo = nullptr;
    bool ms_first = false;
    // timing: 0 off, 1 kernel classes, 2 classes and every lattice-level smoothing pass
    int timing = 0;
    std::vector<TimeRec> recs;
    std::vector<hipEvent_t> pool;
    double tms[EK_T_COUNT] = {0};
    long long tcnt[EK_T_COUNT] = {0};
    double kms[EK_K_COUNT] = {0};      // timing level 3: per kernel
    long long kcnt[EK_K_COUNT] = {0};
    bool in_batch = false;  // owned by a batch: stepping goes through the batch
    // reverse mode (periodic FP64 contexts): checkpoints of the last checkpointed forward
    // run and the adjoint fields
    struct {
        int T = 0, K = 0, nck = 0;  // steps, checkpoint interval, checkpoints (every K steps and the end)
        double* ck = nullptr;       // nck x kCkVals N doubles
        size_t ck_cap = 0;          // checkpoints the allocation holds
        std::vector<double> ck_rate;
        std::vector<long long> ck_steps, ck_ptotal;
        std::vector<int> ck_ws;          // adaptive warm start: order, steps since the probe
        std::vector<double> ck_rel0;     // its last start residuals of orders 2 and 3
        std::vector<int> ck_kring;       // cycles the last solves needed (8 per checkpoint) and
        std::vector<int> ck_kpos;        // the next record's place + 8 x the records held
        double* seg = nullptr;      // K x kSegVals N doubles: the states of one segment
        int seg_cap = 0;
        double* buf = nullptr;      // adjoint fields (kAdjVals N doubles)
        double* gred = nullptr;     // gradient partials per workgroup
        bool valid = false;
    } adj;
    ek_ctx* shadow = nullptr;  // FP64 twin holding the checkpoints of an FP32 context's reverse mode
};

// Checkpoint: populations of a and b (2 x 19 N), stored ions (2 N), the potential and the
// two previous potentials (the warm start of the next solve).  Segment state: populations, ions
// and the potential solved in that step.  Adjoint fields: dL/df (two parities x two
// components x 19 N), dL/dn (two parities x 2 N) and the intermediates of AdjFields.
constexpr size_t kCkVals = 2 * kQ + 5, kSegVals = 2 * kQ + 3, kAdjVals = 4 * kQ + 4 + 6 + 3 + 3 + 2 + 3 + 2 + 1 + 1 + 1 + 2;

#define EK_HIP(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            c->err = std::string(#call) + ": " + hipGetErrorString(e_);                          \
            return EK_EHIP;                                                                      \
        }                                                                                        \
    } while (0)

static ek_status fail(ek_ctx* c, ek_status s, const std::string& msg) {
    c->err = msg;
    return s;
}

static ek_status dalloc(ek_ctx* c, void** ptr, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (c->ws_mode != 0) {  // measure (1) or carve the caller's workspace (2), in 256-byte aligned pieces
        const uintptr_t base = (uintptr_t)c->ws;
        const size_t off = (size_t)((((base + c->ws_used) + 255) & ~(uintptr_t)255) - base);
        if (c->ws_mode == 2 && off + bytes > c->ws_size) {
            c->err = "workspace of " + std::to_string(c->ws_size) + " bytes too small (ek_workspace_bytes)";
            return EK_ENOMEM;
        }
        *ptr = c->ws_mode == 2 ? (void*)(c->ws + off) : nullptr;
        c->ws_used = off + bytes;
        c->bytes += bytes;
        return EK_OK;
    }
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        c->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
        return EK_ENOMEM;
    }
    c->allocs.push_back(*ptr);
    c->bytes += bytes;
    return EK_OK;
}

#define EK_TRY(x)                   \
    do {                            \
        ek_status s_ = (x);         \
        if (s_ != EK_OK) return s_; \
    } while (0)

static void dfree(ek_ctx* c, void* ptr, size_t bytes) {
    if (!ptr) return;
    for (size_t k = 0; k < c->allocs.size(); ++k)
        if (c->allocs[k] == ptr) {  // only buffers from hipMalloc (never a piece of a workspace)
            c->allocs.erase(c->allocs.begin() + (long)k);
            (void)hipFree(ptr);
            c->bytes -= bytes;
            return;
        }
}

// ------------------------------------------------------------------------------------
// Timing (HIP events on the context's stream)
// ------------------------------------------------------------------------------------
constexpr int kKBase = 100;  // Timer classes from here on time single kernels (EK_K_*)

static hipEvent_t get_event(ek_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
}

static void resolve_timing(ek_ctx* c) {
    if (c->recs.empty()) return;
    (void)hipEventSynchronize(c->recs.back().b);
    for (auto& r : c->recs) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        if (r.cls >= kKBase) {
            c->kms[r.cls - kKBase] += ms;
            c->kcnt[r.cls - kKBase] += r.count;
        } else {
            c->tms[r.cls] += ms;
            c->tcnt[r.cls] += r.count;
        }
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
}

struct Timer {
    ek_ctx* c;
    int cls, count;
    hipEvent_t a{};
    bool on;
    // kernel classes at timing levels 1 and 2 (EK_T_SMOOTH only at 2); single kernels
    // (ids kKBase + EK_K_*) only at level 3
    static bool active(const ek_ctx* c, int cls) {
        if (cls >= kKBase) return c->timing == 3;
        if (c->timing == 3) return false;
        return c->timing >= (cls == EK_T_SMOOTH ? 2 : 1);
    }
    Timer(ek_ctx* c_, int cls_, int count_ = 1)
        : c(c_), cls(cls_), count(count_), on(active(c_, cls_)) {
        if (on) {
            a = get_event(c);
            (void)hipEventRecord(a, c->st);
        }
    }
    ~Timer() {
        if (!on) return;
        hipEvent_t b = get_event(c);
        (void)hipEventRecord(b, c->st);
        c->recs.push_back({a, b, cls, count});
        if (c->recs.size() > 4096) resolve_timing(c);
    }
};

// One kernel launch timed at timing level 3.
#define EK_KT(id) Timer kt_##id##__(c, kKBase + (id))

// ------------------------------------------------------------------------------------
// Fields view for one precision
// ------------------------------------------------------------------------------------
template <typename T>
static Fields<T> fields(ek_ctx* c) {
    Fields<T> F;
    for (int k = 0; k < 2; ++k) {
        F.f[k] = (const T*)c->f[c->cur][k];
        F.fn[k] = (T*)c->f[c->cur ^ 1][k];
        F.n[k] = (const T*)c->n[c->cur][k];
        F.nn[k] = (T*)c->n[c->cur ^ 1][k];
    }
    F.mom = (T*)c->mom;
    F.uph = (T*)c->uph;
    F.q = (T*)c->q;
    F.eps = (T*)c->eps;
    F.phi = c->phi;
    F.flags = c->flags;
    F.psif = (const T*)c->psif;
    F.qc = (const T*)c->qc;
    F.owner = c->owner;
    F.linkbase = c->linkbase;
    F.linkdp = c->S.reproject ? nullptr : c->linkdp;  // moving particles: no link lists
    F.vlist = c->vlist;
    F.nv = c->nv;
    F.plist = c->plist;
    F.npl = c->npl;
    F.npl_dev = c->S.reproject ? c->npl_dev : nullptr;
    F.pv = c->pv[c->pcur];
    F.red = c->red;
    F.scal = c->scal;
    F.ms = c->moment_state ? (const T*)c->ms[c->cur] : nullptr;
    F.msn = c->moment_state ? (T*)c->ms[c->cur ^ 1] : nullptr;
    F.rho0 = c->rho0;
    F.ms_first = c->ms_first ? 1 : 0;
    F.rlo = (T*)c->rlo;
    F.mlo = (T*)c->mlo;
    return F;
}

// ------------------------------------------------------------------------------------
// Geometry (host, at set-up): wall layers, particle marking, solid fraction by sub-cell
// counting, charge spreading, boundary lists (Sec. II E).
// ------------------------------------------------------------------------------------
static double wrap_dist(double d, int n) { return min_image(d, n); }

struct HostGeom {
    std::vector<uint8_t> flags;
    std::vector<double> psis, qc;
    std::vector<int32_t> owner, linkbase, vlist, link_off, link_idx, site_off, site_idx;
    std::vector<int32_t> plist;  // sites with flag bits 0, 1 or 3 (the particle path), ascending
    long long nlinks = 0;
};

static ek_status build_geometry(ek_ctx* c, const ek_particle* parts, int np, HostGeom& g) {
    const ek_params& p = c->p;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const size_t N = c->N;
    g.flags.assign(N, 0);
    g.psis.assign(N, 0.0);
    g.qc.assign(N, 0.0);
    g.owner.assign(N, -1);
    auto id = [&](int x, int y, int z) { return (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z); };
    if (p.walls_z) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                g.flags[id(x, y, 0)] |= 1;
                g.flags[id(x, y, nz - 1)] |= 1;
                g.psis[id(x, y, 0)] = 1.0;
                g.psis[id(x, y, nz - 1)] = 1.0;
            }
    }
    const int h = p.subsample > 0 ? p.subsample : 8;
    std::vector<double> offs(h);
    for (int a = 0; a < h; ++a) offs[a] = (a + 0.5) / h - 0.5;
    for (int j = 0; j < np; ++j) {
        const double X = parts[j].x[0], Y = parts[j].x[1], Z = parts[j].x[2], R = parts[j].radius;
        if (!(R > 0.0)) return fail(c, EK_EINVAL, "particle radius must be positive");
        const int lo[3] = {(int)std::floor(X - R) - 1, (int)std::floor(Y - R) - 1, (int)std::floor(Z - R) - 1};
        const int hi[3] = {(int)std::ceil(X + R) + 1, (int)std::ceil(Y + R) + 1, (int)std::ceil(Z + R) + 1};
        for (int zz = lo[2]; zz <= hi[2]; ++zz)
            for (int yy = lo[1]; yy <= hi[1]; ++yy)
                for (int xx = lo[0]; xx <= hi[0]; ++xx) {
                    const int x = ((xx % nx) + nx) % nx, y = ((yy % ny) + ny) % ny, z = ((zz % nz) + nz) % nz;
                    const double dx = wrap_dist((double)x - X, nx), dy = wrap_dist((double)y - Y, ny),
                                 dz = wrap_dist((double)z - Z, nz);
                    int cnt = 0;
                    for (int a = 0; a < h; ++a) {
                        const double sx = dx + offs[a];
                        for (int b = 0; b < h; ++b) {
                            const double sy = dy + offs[b];
                            const double sxy = sx * sx + sy * sy;
                            for (int e = 0; e < h; ++e) {
                                const double sz = dz + offs[e];
                                if (sxy + sz * sz <= R * R) ++cnt;
                            }
                        }
                    }
                    const size_t i = id(x, y, z);
                    const bool wall = p.walls_z && (z == 0 || z == nz - 1);
                    if (cnt > 0 && !wall) {
                        if (g.owner[i] >= 0 && g.owner[i] != j)
                            return fail(c, EK_EINVAL, "particles overlap on the lattice");
                        g.owner[i] = j;
                        g.psis[i] = (double)cnt / ((double)h * h * h);
                    }
                    if (dx * dx + dy * dy + dz * dz < R * R) g.flags[i] |= 1;
                }
    }
    if (np > 0) {
        std::vector<double> tot(np, 0.0);
        for (size_t i = 0; i < N; ++i)
            if (g.owner[i] >= 0) tot[g.owner[i]] += g.psis[i];
        for (size_t i = 0; i < N; ++i)
            if (g.owner[i] >= 0 && tot[g.owner[i]] > 0.0) g.qc[i] = parts[g.owner[i]].charge * g.psis[i] / tot[g.owner[i]];
    }
    // neighbour flags, virtual-density list, particle links
    g.linkbase.assign(np > 0 ? N : 1, 0);
    long long nl = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t i = id(x, y, z);
                const bool si = g.flags[i] & 1;
                bool any_other = false;
                int links_here = 0;
                for (int d = 0; d < kQ; ++d) {
                    if (d == kRest) continue;
                    const size_t j = id(((x + vx(d)) % nx + nx) % nx, ((y + vy(d)) % ny + ny) % ny,
                                        ((z + vz(d)) % nz + nz) % nz);
                    const bool sj = g.flags[j] & 1;
                    if (sj != si) any_other = true;
                    if (!si && sj && g.owner[j] >= 0) ++links_here;
                }
                if (any_other) g.flags[i] |= si ? 4 : 2;
                if (si && any_other) g.vlist.push_back((int32_t)i);
                if (np > 0 && links_here) {
                    g.linkbase[i] = (int32_t)nl;
                    nl += links_here;
                }
            }
    g.nlinks = nl;
    // bit 3: the site or one of its six axis neighbours is partly covered (fluid fraction
    // below 1).  A site with none of bits 0, 1 and 3 sees fluid fraction 1 and no solid
    // around it, and the stencil passes take the plain path there.
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t i = id(x, y, z);
                bool part = g.psis[i] > 0.0;
                for (int k = 0; k < 3 && !part; ++k)
                    for (int sgn = -1; sgn <= 1 && !part; sgn += 2) {
                        const size_t j = id(((x + (k == 0 ? sgn : 0)) % nx + nx) % nx,
                                            ((y + (k == 1 ? sgn : 0)) % ny + ny) % ny,
                                            ((z + (k == 2 ? sgn : 0)) % nz + nz) % nz);
                        part = g.psis[j] > 0.0;
                    }
                if (part) g.flags[i] |= 8;
            }
    if (np > 0)
        for (size_t i = 0; i < N; ++i)
            if (g.flags[i] & (1 | 2 | 8)) g.plist.push_back((int32_t)i);
    if (np > 0) {
        // links grouped by particle (counting sort), in the order the fused kernel writes them
        std::vector<int32_t> lowner(nl > 0 ? nl : 1);
        long long l = 0;
        for (size_t i = 0; i < N; ++i) {
            if ((g.flags[i] & 1) || !(g.flags[i] & 2)) continue;
            const int x = i % nx, y = (i / nx) % ny, z = i / ((size_t)nx * ny);
            for (int d = 0; d < kQ; ++d) {
                if (d == kRest) continue;
                const size_t j = id(((x + vx(d)) % nx + nx) % nx, ((y + vy(d)) % ny + ny) % ny,
                                    ((z + vz(d)) % nz + nz) % nz);
                if ((g.flags[j] & 1) && g.owner[j] >= 0) lowner[l++] = g.owner[j];
            }
        }
        g.link_off.assign(np + 1, 0);
        for (long long t = 0; t < nl; ++t) g.link_off[lowner[t] + 1]++;
        for (int j = 0; j < np; ++j) g.link_off[j + 1] += g.link_off[j];
        g.link_idx.assign(nl > 0 ? nl : 1, 0);
        std::vector<int32_t> fill(g.link_off.begin(), g.link_off.end() - 1);
        for (long long t = 0; t < nl; ++t) g.link_idx[fill[lowner[t]]++] = (int32_t)t;
        g.site_off.assign(np + 1, 0);
        for (size_t i = 0; i < N; ++i)
            if (g.owner[i] >= 0) g.site_off[g.owner[i] + 1]++;
        for (int j = 0; j < np; ++j) g.site_off[j + 1] += g.site_off[j];
        g.site_idx.assign(std::max<int32_t>(g.site_off[np], 1), 0);
        std::vector<int32_t> sf(g.site_off.begin(), g.site_off.end() - 1);
        for (size_t i = 0; i < N; ++i)
            if (g.owner[i] >= 0) g.site_idx[sf[g.owner[i]]++] = (int32_t)i;
    }
    return EK_OK;
}

// ------------------------------------------------------------------------------------
// Poisson solve with convergence control
// ------------------------------------------------------------------------------------
// The fewest V-cycles any of the last (up to eight) own multigrid solves needed; 0 when none
// is recorded (at set-up, or after a change of the cycle shape).
static int cycles_floor(const ek_ctx* c) {
    if (c->kcount == 0) return 0;
    int m = c->kring[0];
    for (int k = 1; k < c->kcount; ++k) m = std::min(m, c->kring[k]);
    return m;
}
static void cycles_record(ek_ctx* c, int k) {
    c->kring[c->kpos] = k;
    c->kpos = (c->kpos + 1) % 8;
    c->kcount = std::min(c->kcount + 1, 8);
}
static void cycles_forget(ek_ctx* c) {
    for (int k = 0; k < 8; ++k) c->kring[k] = 0;
    c->kpos = 0;
    c->kcount = 0;
}

// F in site order (split false) and pack: the kernel also fills c->phis, c->qs.
template <typename T>
static ek_status check_residual(ek_ctx* c, const Fields<T>& F, bool split, bool pack, double& rr, double& ss) {
    const unsigned nres = residual_blocks(c->N);
    {
        EK_KT(EK_K_RESIDUAL);
        launch_residual<T>(c->S, F, nres, split, pack ? c->phis : nullptr, pack ? (T*)c->qs : nullptr, c->st);
    }
    {
        EK_KT(EK_K_REDUCE);
        launch_reduce(c->red, nres, 3, nullptr, c->scal + 1, c->st);
    }
    EK_HIP(hipMemcpyAsync(c->hscal, c->scal, 4 * sizeof(double), hipMemcpyDeviceToHost, c->st));
    EK_HIP(hipStreamSynchronize(c->st));
    rr = c->hscal[1];
    ss = c->hscal[2];
    c->last_mean = c->hscal[0];
    return EK_OK;
}

// One V-cycle on the lattice (grid 0) with the coarse grids c->mg[0..nl-1] (grid g >= 1 is
// c->mg[g - 1]).  The last one or two grids are handled by the single-workgroup tail
// kernel (the coarsest solve, and the sweeps of the grid above it when small enough).
// split: F holds the colour-split lattice potential and charge.
template <typename T>
static void vcycle(ek_ctx* c, const Fields<T>& F0, bool split) {
    const int nl = (int)c->mg.size();
    const int tail_mid = (nl >= 2 && c->mg[nl - 2].n <= 4096 && c->mg[nl - 1].n <= 512) ? 1 : 0;
    const int last_gpu = nl - 1 - tail_mid;  // finest grid handled by the tail, minus one
    // F.phi: the buffer that holds the lattice potential.  On colour-split fields a lattice
    // sweep runs in one pass (k_sor_rb) from one buffer to the other (F0.phi, c->stage)
    // where the kernel fits; an even number of such sweeps per cycle, so that the cycle
    // ends in F0.phi, and the rest as two colour passes in place.
    Fields<T> F = F0;
    const bool rb = split && c->one_pass && sor_rb_fits(c->S);
    int rb_left = rb ? c->mg_fine_pre + c->mg_fine_post - (c->mg_fine_post >= 1 ? 1 : 0) : 0;
    rb_left -= rb_left & 1;
    // multigrid grids have even axes: two colours; first = 1 skips the red pass (taken by the
    // restriction into a launched coarse grid)
    auto smooth = [&](int g, int first = 0) {
        if (g == 0 && first == 0 && rb_left > 0) {
            double* to = F.phi == F0.phi ? c->stage : F0.phi;
            EK_KT(EK_K_SOR_RB);
            launch_sor_rb<T>(c->S, F, F.phi, to, c->mg_omega, c->st);
            F.phi = to;
            --rb_left;
            return;
        }
        for (int color = first; color < 2; ++color) {
            if (g == 0) {
                EK_KT(EK_K_SOR);
                launch_sor<T>(c->S, F, color, c->mg_omega, split, c->st);
            } else {
                EK_KT(EK_K_SMOOTH);
                launch_mg_smooth(c->mg[g - 1], color, c->mg_omega, c->st);
            }
        }
    };
    // the lattice sweeps of one leg run back to back: one event pair times the group
    auto smooth_lattice = [&](int sweeps) {
        if (sweeps <= 0) return;
        Timer tm(c, EK_T_SMOOTH, 2 * sweeps);
        for (int s = 0; s < sweeps; ++s) smooth(0);
    };
    // the restriction into a launched coarse grid takes that grid's first red pass
    const double red = c->mg_pre >= 1 ? c->mg_omega : 0.0;
    for (int g = 0; g <= last_gpu; ++g) {  // downward leg: smooth grid g, restrict to grid g+1
        const int pre = g == 0 ? c->mg_fine_pre : c->mg_pre;
        if (g == 0)
            smooth_lattice(pre);
        else
            for (int s = 0; s < pre; ++s) smooth(g, s == 0 && red > 0.0 ? 1 : 0);
        const double r = g + 1 <= last_gpu ? red : 0.0;
        if (g == 0) {
            EK_KT(EK_K_RESTRICT_FINE);
            launch_mg_restrict_fine<T>(c->S, F, c->mg[0], split, r, c->st);
        } else {
            EK_KT(EK_K_RESTRICT);
            launch_mg_restrict(c->mg[g - 1], c->mg[g], r, c->st);
        }
    }
    {
        EK_KT(EK_K_TAIL);
        launch_mg_tail(tail_mid ? c->mg[nl - 2] : c->mg[nl - 1], c->mg[nl - 1], tail_mid, c->mg_coarsest,
                       c->mg_coarse_omega, c->mg_tail_pre, c->mg_tail_post, c->mg_omega, c->st);
    }
    for (int g = last_gpu; g >= 0; --g) {  // upward leg: interpolate from grid g+1, smooth grid g
        const int post = g == 0 ? c->mg_fine_post : c->mg_post;
        if (g == 0 && split && post >= 1) {
            // colour-split lattice: the interpolation takes the first red pass, and the black
            // pass reads the interpolated black values from c->blk
            {
                EK_KT(EK_K_PROLONG_RED_FINE);
                launch_mg_prolong_red_fine<T>(c->S, F, c->mg[0], c->mg_omega, c->blk, c->st);
            }
            Timer tm(c, EK_T_SMOOTH, 2 * post - 1);
            {
                EK_KT(EK_K_SOR_BLACK_FROM);
                launch_sor_black_from<T>(c->S, F, c->mg_omega, c->blk, c->st);
            }
            for (int s = 1; s < post; ++s) smooth(0);
            continue;
        }
        if (g == 0) {
            EK_KT(EK_K_PROLONG_FINE);
            launch_mg_prolong_fine<T>(c->S, F, c->mg[0], split, c->st);
        } else {
            EK_KT(EK_K_PROLONG);
            launch_mg_prolong(c->mg[g], c->mg[g - 1], c->st);
        }
        if (g == 0)
            smooth_lattice(post);
        else
            for (int s = 0; s < post; ++s) smooth(g);
    }
}

static void vcycle_graph_drop(ek_ctx* c) {
    if (c->vc_exec) (void)hipGraphExecDestroy(c->vc_exec);
    if (c->vc_graph) (void)hipGraphDestroy(c->vc_graph);
    c->vc_exec = nullptr;
    c->vc_graph = nullptr;
}

// A solve of the context's own potential and charge, or the reverse sweep's adjoint solve.
static bool own_solve(const ek_ctx* c) {
    return (c->phi == c->phi_own && c->q == c->q_own) || c->adj_solve;
}

// k V-cycles: graph replays when possible, direct launches otherwise.  The graph is
// captured (and replayed) only for the context's own potential and charge, in the layout
// (colour-split or site order) it was captured with.
template <typename T>
static ek_status run_cycles(ek_ctx* c, Fields<T>& F, bool split, int k) {
    const bool own = own_solve(c);
    if (own && c->vc_exec && c->vc_split != split) vcycle_graph_drop(c);  // other solves launch directly
    if (c->timing < 2 && own && !c->vc_off && !c->vc_exec) {
        if (!c->cap_st) EK_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
        hipStream_t st = c->st;
        c->st = c->cap_st;
        bool ok = hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            vcycle<T>(c, F, split);
            c->vc_split = split;
            ok = hipStreamEndCapture(c->cap_st, &c->vc_graph) == hipSuccess;
        }
        c->st = st;
        if (ok) ok = hipGraphInstantiate(&c->vc_exec, c->vc_graph, nullptr, nullptr, 0) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            vcycle_graph_drop(c);
            c->vc_off = true;  // this runtime cannot capture the cycle: launch it directly from now on
        }
    }
    if (c->vc_exec && c->timing < 2 && own) {
        for (int s = 0; s < k; ++s) EK_HIP(hipGraphLaunch(c->vc_exec, c->st));
    } else {
        for (int s = 0; s < k; ++s) vcycle<T>(c, F, split);
    }
    return EK_OK;
}

// Coarse-level face coefficients for the current permittivity.
template <typename T>
static void mg_build(ek_ctx* c, const Fields<T>& F) {
    {
        EK_KT(EK_K_COARSEN);
        launch_mg_coarsen_fine<T>(c->S, F, c->mg[0], c->st);
    }
    for (size_t l = 1; l < c->mg.size(); ++l) {
        EK_KT(EK_K_COARSEN);
        launch_mg_coarsen(c->mg[l - 1], c->mg[l], c->st);
    }
}

// Requires q, eps and the source mean of the current state on the device.
template <typename T>
static ek_status poisson_solve(ek_ctx* c, double tol, int maxit, int* iters_out, double* rel_out, bool fixed = false) {
    Timer tm(c, EK_T_POISSON);
    Fields<T> F = fields<T>(c);
    const bool use_mg = !c->mg.empty();
    const bool own = own_solve(c);
    // a multigrid solve of the context's own potential runs on colour-split copies of the
    // potential and charge; the gauge kernel writes the result back in site order
    const bool split = c->phis && use_mg && own;
    Fields<T> FS = F;
    if (split) {
        FS.phi = c->phis;
        FS.q = (T*)c->qs;
    }
    if (fixed && use_mg && own) {
        // A fixed number of V-cycles and no host read-back: the start and end residuals are
        // reduced on the device, where ek_observables reads them (and the largest since its
        // last call).  The step is then one stream of launches with no synchronisation.
        const int k = c->fixed_cycles;
        const unsigned nres = residual_blocks(c->N);
        {
            EK_KT(EK_K_RESIDUAL);
            launch_residual<T>(c->S, F, nres, false, split ? c->phis : nullptr, split ? (T*)c->qs : nullptr, c->st);
        }
        {
            EK_KT(EK_K_REDUCE);
            launch_reduce(c->red, nres, 3, nullptr, c->scal + 24, c->st);
        }
        mg_build<T>(c, F);
        {
            Timer ts(c, EK_T_ITER, k);
            EK_TRY(run_cycles<T>(c, FS, split, k));
        }
        {
            EK_KT(EK_K_RESIDUAL);
            launch_residual<T>(c->S, FS, nres, split, nullptr, nullptr, c->st);
        }
        {
            EK_KT(EK_K_REDUCE);
            launch_reduce(c->red, nres, 3, nullptr, c->scal + 1, c->st);
        }
        launch_track_residual(c->scal, c->st);
        {
            EK_KT(EK_K_FINALIZE);
            launch_phi_finalize<T>(c->S, F, 0, split ? c->phis : nullptr, c->st);
        }
        EK_HIP(hipGetLastError());
        c->last_iters = k;
        c->ptotal += k;
        if (iters_out) *iters_out = k;
        if (rel_out) *rel_out = -1.0;
        return EK_OK;
    }
    // the cycle rate: geometric mean over the last k cycles, kept on the slow side
    auto update_rate = [&](double r_old, double r_new, int k) {
        if (r_new < r_old && r_new > 0.0) {
            const double est = std::pow(r_new / r_old, 1.0 / k);
            c->rate = c->rate > 0.0 ? std::max(est, 0.5 * (c->rate + est)) : est;
        }
    };
    // Multigrid solves of the context's own potential launch the cycles that every one of
    // the last solves needed (k0) before reading back the first residual: one host round
    // trip fewer per solve.  The first check's sums go to scal[24..26].
    const int k0 = own && use_mg ? std::min(cycles_floor(c), maxit) : 0;
    double rr, ss, r_k0 = 0.0;
    int it = 0;
    bool built = false;
    if (k0 > 0) {
        const unsigned nres = residual_blocks(c->N);
        {
            EK_KT(EK_K_RESIDUAL);
            launch_residual<T>(c->S, F, nres, false, split ? c->phis : nullptr, split ? (T*)c->qs : nullptr, c->st);
        }
        {
            EK_KT(EK_K_REDUCE);
            launch_reduce(c->red, nres, 3, nullptr, c->scal + 24, c->st);
        }
        mg_build<T>(c, F);
        built = true;
        {
            Timer ts(c, EK_T_ITER, k0);
            EK_TRY(run_cycles<T>(c, FS, split, k0));
        }
        EK_HIP(hipGetLastError());
        it = k0;
        {
            EK_KT(EK_K_RESIDUAL);
            launch_residual<T>(c->S, FS, nres, split, nullptr, nullptr, c->st);
        }
        {
            EK_KT(EK_K_REDUCE);
            launch_reduce(c->red, nres, 3, nullptr, c->scal + 1, c->st);
        }
        EK_HIP(hipMemcpyAsync(c->hscal, c->scal, 4 * sizeof(double), hipMemcpyDeviceToHost, c->st));
        EK_HIP(hipMemcpyAsync(c->hscal + 24, c->scal + 24, 3 * sizeof(double), hipMemcpyDeviceToHost, c->st));
        EK_HIP(hipStreamSynchronize(c->st));
        rr = c->hscal[24];
        ss = c->hscal[25];
        r_k0 = std::sqrt(c->hscal[1]);
        c->last_mean = c->hscal[0];
    } else {
        EK_TRY(check_residual<T>(c, F, false, split, rr, ss));  // from site order, filling the split copies
    }
    c->last_rel0 = ss > 0.0 ? std::sqrt(rr / ss) : 0.0;
    ek_status status = EK_OK;
    double rel = 0.0;
    int need = 0;  // cycles this solve needed (for the next solves' k0)
    if (!(ss > 0.0)) {
        EK_KT(EK_K_FINALIZE);
        launch_phi_finalize<T>(c->S, F, 1, nullptr, c->st);
    } else {
        const double target = tol * std::sqrt(ss);
        const double r0 = std::sqrt(rr);
        double r = r0;
        if (k0 > 0) {
            update_rate(r, r_k0, k0);
            r = r_k0;
        }
        if (use_mg && r > target && !built) mg_build<T>(c, F);
        while (use_mg && r > target && it < maxit) {
            int k = 1;
            if (c->rate > 0.0 && c->rate < 1.0) k = (int)std::ceil(std::log(target / r) / std::log(c->rate));
            k = std::max(1, std::min(k, 8));
            k = std::min(k, maxit - it);
            {
                Timer ts(c, EK_T_ITER, k);
                EK_TRY(run_cycles<T>(c, FS, split, k));
            }
            EK_HIP(hipGetLastError());
            it += k;
            EK_TRY(check_residual<T>(c, FS, split, false, rr, ss));
            const double rn = std::sqrt(rr);
            update_rate(r, rn, k);
            r = rn;
        }
        while (!use_mg && r > target && it < maxit) {
            int k;
            if (c->rate > 0.0 && c->rate < 1.0)
                k = (int)std::ceil(1.1 * std::log(target / r) / std::log(c->rate)) + 1;
            else
                k = 8;
            k = std::max(1, std::min(k, 400));
            k = std::min(k, maxit - it);
            {
                Timer ts(c, EK_T_ITER, k);
                Timer tm(c, EK_T_SMOOTH, c->S.ncolor * k);  // the k sweeps run back to back
                for (int s = 0; s < k; ++s)
                    for (int color = 0; color < c->S.ncolor; ++color) {
                        EK_KT(EK_K_SOR);
                        launch_sor<T>(c->S, F, color, c->omega, false, c->st);
                    }
            }
            EK_HIP(hipGetLastError());
            it += k;
            EK_TRY(check_residual<T>(c, FS, split, false, rr, ss));
            const double rn = std::sqrt(rr);
            update_rate(r, rn, k);
            r = rn;
        }
        {
            EK_KT(EK_K_FINALIZE);
            launch_phi_finalize<T>(c->S, F, 0, split ? c->phis : nullptr, c->st);
        }
        rel = r / std::sqrt(ss);
        if (r > target) status = EK_ENOCONV;
        // cycles needed: the first count at which the solve's mean decay per cycle reaches
        // the target (at most the cycles run), so that running k0 cycles does not lock k0 in
        need = it;
        if (r0 <= target) {
            need = 0;
        } else if (it > 0 && r > 0.0 && r < r0) {
            const double rho = std::pow(r / r0, 1.0 / it);
            need = std::min(it, std::max(0, (int)std::ceil(std::log(target / r0) / std::log(rho) - 1e-9)));
        }
    }
    EK_HIP(hipGetLastError());
    if (own && use_mg) cycles_record(c, need);
    c->last_iters = it;
    c->last_rel = rel;
    c->rel_max = std::max(c->rel_max, rel);
    c->ptotal += it;
    if (iters_out) *iters_out = it;
    if (rel_out) *rel_out = rel;
    if (status == EK_ENOCONV) c->err = "Poisson solve stopped at maxit above the tolerance";
    return status;
}

template <typename T>
static void moments_pass(ek_ctx* c) {
    Timer tm(c, EK_T_MOMENTS);
    Fields<T> F = fields<T>(c);
    {
        EK_KT(EK_K_MOMENTS);
        launch_moments<T>(c->S, F, c->nblk, c->st);
    }
    {
        EK_KT(EK_K_VIRTUAL);
        launch_virtual<T>(c->S, F, c->st);
    }
    EK_KT(EK_K_SOURCE_MEAN);
    launch_source_mean(c->S, c->red, c->nblk, c->scal, c->st);
}

// The rest of a step after the Poisson solve: forces, the fused sweep, particles, and the
// swap of the step parity.
template <typename T>
static ek_status step_rest(ek_ctx* c) {
    Fields<T> F = fields<T>(c);
    {
        Timer tm(c, EK_T_FORCE);
        EK_KT(EK_K_FORCE);
        launch_force<T>(c->S, F, c->st);
    }
    {
        Timer tm(c, EK_T_FUSED);
        EK_KT(EK_K_FUSED);
        launch_fused<T>(c->S, F, c->st);
    }
    if (c->np > 0) {
        Timer tm(c, EK_T_PARTICLE);
        EK_KT(EK_K_PARTICLE);
        launch_particle_step<T>(c->S, F, c->np, c->plink_off, c->plink_idx, c->psite_off, c->psite_idx,
                                c->px[c->pcur], c->pv[c->pcur], c->prad, c->pF, c->px[c->pcur ^ 1],
                                c->pv[c->pcur ^ 1], c->p.particle_rho, c->p.k_hertz, c->p.eta, c->p.move_particles,
                                c->st);
        c->pcur ^= 1;
    }
    if (c->S.reproject) {
        Timer tm(c, EK_T_PARTICLE);
        EK_KT(EK_K_REPROJECT);
        const size_t N = c->N;
        EK_HIP(hipMemcpyAsync(c->flags_old, c->flags, N, hipMemcpyDeviceToDevice, c->st));
        EK_HIP(hipMemcpyAsync(c->owner_old, c->owner, N * 4, hipMemcpyDeviceToDevice, c->st));
        EK_HIP(hipMemcpyAsync(c->psif_old, c->psif, N * c->esz, hipMemcpyDeviceToDevice, c->st));
        Reproj<T> P{c->np, c->px[c->pcur], c->pv[c->pcur], c->prad, c->pQ, c->p.particle_rho, c->flags, c->owner,
                    (T*)c->psif, (T*)c->qc, c->flags_old, c->owner_old, (const T*)c->psif_old, c->rp_origin,
                    c->rp_cnt, c->rp_inside, c->rp_event, c->rp_evm, (T*)c->rp_share, c->rp_ptot, c->rp_nb, c->rp_nnb,
                    c->plist, c->npl_dev};
        launch_reproject<T>(c->S, F, P, c->st);
    }
    EK_HIP(hipGetLastError());
    c->cur ^= 1;
    c->ms_first = false;  // a moment-state context now holds the state written by this step
    c->steps++;
    return EK_OK;
}

// One lagged Fourier solve (ek_fft.hip) from the potential held: right-hand side, forward
// FFT, spectral division, inverse FFT into the potential.
template <typename T>
static ek_status lagged_fourier(ek_ctx* c) {
    Timer tm(c, EK_T_POISSON);
    EK_KT(EK_K_LAGGED);
    launch_lag_rhs<T>(c->S, fields<T>(c), c->fft_rhs, c->st);
    if (hipfftExecD2Z(c->fft_fwd, c->fft_rhs, (hipfftDoubleComplex*)c->fft_spec) != HIPFFT_SUCCESS)
        return fail(c, EK_EHIP, "hipfftExecD2Z failed");
    launch_lag_scale(c->fft_spec, c->fft_tab, c->S.nx, c->S.ny, c->S.nz, c->st);
    if (hipfftExecZ2D(c->fft_inv, (hipfftDoubleComplex*)c->fft_spec, c->phi) != HIPFFT_SUCCESS)
        return fail(c, EK_EHIP, "hipfftExecZ2D failed");
    EK_HIP(hipGetLastError());
    c->last_iters = 1;
    c->last_rel = -1.0;  // not measured (it would cost a residual pass and a host read-back per step)
    c->ptotal += 1;
    return EK_OK;
}

template <typename T>
static ek_status step_impl(ek_ctx* c, int nsteps) {
    ek_status worst = EK_OK;
    for (int s = 0; s < nsteps; ++s) {
        moments_pass<T>(c);
        if (c->fft) {
            EK_TRY(lagged_fourier<T>(c));
            EK_TRY(step_rest<T>(c));
            continue;
        }
        const bool fixed = c->fixed_cycles > 0;
        int order = c->phi_history;
        bool probe = false;
        if (order == 0 && fixed) order = 2;  // the adaptive choice needs the start residuals on the host
        if (order == 0) {  // adaptive: keep the order with the smaller start residual, re-probe the other
            order = c->ws_order;
            const int other = 5 - c->ws_order;
            if (c->rel0_of[c->ws_order] > 0.0 && (c->rel0_of[other] == 0.0 || c->ws_since >= 64)) {
                order = other;
                probe = true;
            }
        }
        {
            EK_KT(EK_K_EXTRAPOLATE);
            launch_phi_extrapolate(c->S, c->phi, c->phi_prev, c->phi_prev2, order, c->st);
        }
        ek_status ps = poisson_solve<T>(c, c->p.poisson_tol, c->p.poisson_maxit, nullptr, nullptr, fixed);
        if (c->phi_history == 0 && !fixed && c->steps >= 2) {
            c->rel0_of[order] = c->last_rel0;
            const int other = 5 - order;
            if (probe) {
                c->ws_since = 0;
                if (c->rel0_of[order] < c->rel0_of[other]) c->ws_order = order;
            } else {
                ++c->ws_since;
            }
        }
        if (ps == EK_ENOCONV)
            worst = ps;
        else if (ps != EK_OK)
            return ps;
        EK_TRY(step_rest<T>(c));
    }
    return worst;
}

// ------------------------------------------------------------------------------------
// Public ABI
// ------------------------------------------------------------------------------------
extern "C" int32_t ek_lattice(int32_t* cvec, double* w) {
    for (int d = 0; d < kQ; ++d) {
        if (cvec) {
            cvec[3 * d] = vx(d);
            cvec[3 * d + 1] = vy(d);
            cvec[3 * d + 2] = vz(d);
        }
        if (w) w[d] = weight(d);
    }
    return kQ;
}

extern "C" double ek_min_image(double d, int32_t n) { return n > 0 ? min_image(d, n) : NAN; }

static double omega_for(const ek_params& p) {
    const double pi = 3.14159265358979323846;
    double lam = 1e300;
    int act = 0;
    if (p.nx > 1) {
        lam = std::min(lam, 2.0 - 2.0 * std::cos(2.0 * pi / p.nx));
        ++act;
    }
    if (p.ny > 1) {
        lam = std::min(lam, 2.0 - 2.0 * std::cos(2.0 * pi / p.ny));
        ++act;
    }
    if (p.walls_z) {
        if (p.nz - 2 > 1) {
            lam = std::min(lam, 2.0 - 2.0 * std::cos(pi / (p.nz - 2)));
            ++act;
        }
    } else if (p.nz > 1) {
        lam = std::min(lam, 2.0 - 2.0 * std::cos(2.0 * pi / p.nz));
        ++act;
    }
    if (act == 0) return 1.0;
    const double mu = 1.0 - lam / (2.0 * act);
    return 2.0 / (1.0 + std::sqrt(std::max(0.0, 1.0 - mu * mu)));
}

// Every device buffer of a context, in one place.  With c->ws_mode 0 each comes from
// hipMalloc; with 1 the sizes are only added up (ek_workspace_bytes, no device call); with 2
// they are carved from the caller's workspace.  Buffers created later (checkpoints, the
// autotuner's state copy, a moment-state population export) always come from hipMalloc.
template <typename T>
static ek_status allocate_all(ek_ctx* c, const HostGeom& g, int np) {
    const ek_params& p = c->p;
    const unsigned N = c->N;
    const size_t es = sizeof(T);
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 2; ++k) {
            if (!c->moment_state) EK_TRY(dalloc(c, &c->f[b][k], (size_t)kQ * N * es));
            EK_TRY(dalloc(c, &c->n[b][k], (size_t)N * es));
        }
    if (c->moment_state) {
        for (int b = 0; b < 2; ++b) EK_TRY(dalloc(c, &c->ms[b], 8 * (size_t)N * es));
        EK_TRY(dalloc(c, (void**)&c->rho0, 2 * (size_t)N * 8));
    }
    if (es == 4 && !c->moment_state && !p.fp32_plain_collision) {
        EK_TRY(dalloc(c, &c->rlo, 2 * (size_t)N * es));
        EK_TRY(dalloc(c, &c->mlo, 2 * (size_t)N * es));
    }
    EK_TRY(dalloc(c, &c->mom, 8 * (size_t)N * es));
    EK_TRY(dalloc(c, &c->uph, 3 * (size_t)N * es));
    EK_TRY(dalloc(c, &c->q, (size_t)N * es));
    EK_TRY(dalloc(c, &c->eps, (size_t)N * es));
    EK_TRY(dalloc(c, (void**)&c->phi, (size_t)N * 8));
    EK_TRY(dalloc(c, (void**)&c->phi_prev, (size_t)N * 8));
    EK_TRY(dalloc(c, (void**)&c->phi_prev2, (size_t)N * 8));
    if (c->split_layout) {
        EK_TRY(dalloc(c, (void**)&c->phis, (size_t)N * 8));
        EK_TRY(dalloc(c, &c->qs, (size_t)N * es));
        EK_TRY(dalloc(c, (void**)&c->blk, (size_t)(N / 2) * 8));
    }
    EK_TRY(dalloc(c, (void**)&c->red, (size_t)c->nblk * kRedSlots * 8));
    EK_TRY(dalloc(c, (void**)&c->scal, 32 * 8));
    EK_TRY(dalloc(c, (void**)&c->obs_max, 16 * sizeof(int)));
    EK_TRY(dalloc(c, (void**)&c->stage, (size_t)N * 8));
    EK_TRY(dalloc(c, (void**)&c->stage2, (size_t)N * 8));
    for (auto& L : c->mg) {
        EK_TRY(dalloc(c, (void**)&L.phi, (size_t)L.n * 8));
        EK_TRY(dalloc(c, (void**)&L.s, (size_t)L.n * 8));
        EK_TRY(dalloc(c, (void**)&L.ax, (size_t)L.n * 8));
        EK_TRY(dalloc(c, (void**)&L.ay, (size_t)L.n * 8));
        EK_TRY(dalloc(c, (void**)&L.az, (size_t)L.n * 8));
    }
    if (!g.vlist.empty()) EK_TRY(dalloc(c, (void**)&c->vlist, g.vlist.size() * 4));
    if (c->S.reproject) {  // room for every box site (the particle-path sites all lie in the boxes)
        const size_t B3 = (size_t)c->S.rp_box * c->S.rp_box * c->S.rp_box;
        const size_t cap = std::max(g.plist.size(), std::min((size_t)N, (size_t)np * B3));
        EK_TRY(dalloc(c, (void**)&c->plist, cap * 4));
        EK_TRY(dalloc(c, (void**)&c->npl_dev, 4));
    } else if (!g.plist.empty()) {
        EK_TRY(dalloc(c, (void**)&c->plist, g.plist.size() * 4));
    }
    if (np > 0) {
        EK_TRY(dalloc(c, (void**)&c->flags, N));
        EK_TRY(dalloc(c, &c->psif, (size_t)N * es));
        EK_TRY(dalloc(c, &c->qc, (size_t)N * es));
        EK_TRY(dalloc(c, (void**)&c->owner, (size_t)N * 4));
        EK_TRY(dalloc(c, (void**)&c->linkbase, (size_t)N * 4));
        EK_TRY(dalloc(c, (void**)&c->linkdp, (size_t)std::max(1LL, g.nlinks) * 6 * 8));
        EK_TRY(dalloc(c, (void**)&c->plink_off, g.link_off.size() * 4));
        EK_TRY(dalloc(c, (void**)&c->plink_idx, g.link_idx.size() * 4));
        EK_TRY(dalloc(c, (void**)&c->psite_off, g.site_off.size() * 4));
        EK_TRY(dalloc(c, (void**)&c->psite_idx, g.site_idx.size() * 4));
        for (int b = 0; b < 2; ++b) {
            EK_TRY(dalloc(c, (void**)&c->px[b], 3 * np * 8));
            EK_TRY(dalloc(c, (void**)&c->pv[b], 3 * np * 8));
        }
        EK_TRY(dalloc(c, (void**)&c->prad, np * 8));
        EK_TRY(dalloc(c, (void**)&c->pF, 3 * np * 8));
        if (c->S.reproject) {
            const size_t B3 = (size_t)c->S.rp_box * c->S.rp_box * c->S.rp_box;
            EK_TRY(dalloc(c, (void**)&c->pQ, np * 8));
            EK_TRY(dalloc(c, (void**)&c->flags_old, N));
            EK_TRY(dalloc(c, (void**)&c->owner_old, (size_t)N * 4));
            EK_TRY(dalloc(c, &c->psif_old, (size_t)N * es));
            EK_TRY(dalloc(c, (void**)&c->rp_origin, 3 * np * 4));
            EK_TRY(dalloc(c, (void**)&c->rp_nb, np * np * 4));
            EK_TRY(dalloc(c, (void**)&c->rp_nnb, np * 4));
            EK_TRY(dalloc(c, (void**)&c->rp_cnt, np * B3 * 2));
            EK_TRY(dalloc(c, (void**)&c->rp_inside, np * B3));
            EK_TRY(dalloc(c, (void**)&c->rp_event, np * B3));
            EK_TRY(dalloc(c, (void**)&c->rp_evm, 3 * np * B3 * 8));
            EK_TRY(dalloc(c, &c->rp_share, (size_t)2 * N * es));
            EK_TRY(dalloc(c, (void**)&c->rp_ptot, np * 8));
        }
    }
    if (c->fft) {
        EK_TRY(dalloc(c, (void**)&c->fft_rhs, (size_t)N * 8));
        EK_TRY(dalloc(c, (void**)&c->fft_spec, (size_t)p.nz * p.ny * (p.nx / 2 + 1) * 16));
        EK_TRY(dalloc(c, (void**)&c->fft_tab, (size_t)(p.nx / 2 + 1 + p.ny + p.nz) * 8));
    }
    return EK_OK;
}

// Reference densities of the FP32 deviation storage, unless given.  A stored deviation
// rho - r carries a rounding error proportional to |rho - r|, so the relative error of rho
// scales with |rho - r| / rho.  Over the initial range [lo, hi] of a component the worst case
// of that ratio is smallest for the harmonic mean r = 2 lo hi / (lo + hi): near the mean for
// a nearly uniform fluid, near the minority value of a demixed one (where a plain mean would
// cost the minority phase two decades of precision).
static ek_status reference_densities(ek_ctx* c, const HostGeom& g, const double* rho_a, const double* rho_b,
                                     const double* n_plus, const double* n_minus) {
    const unsigned N = c->N;
    for (int s = 0; s < 2; ++s) {
        const double* r = s == 0 ? rho_a : rho_b;
        double lo = INFINITY, hi = 0.0;
        for (unsigned i = 0; i < N; ++i) {
            if (g.flags[i] & 1) continue;
            if (!(r[i] > 0.0) || !std::isfinite(r[i])) return fail(c, EK_EINVAL, "fluid densities must be positive and finite");
            lo = std::min(lo, r[i]);
            hi = std::max(hi, r[i]);
        }
        c->S.rref[s] = c->p.rho_ref[s] > 0.0 ? c->p.rho_ref[s] : (hi > 0.0 ? 2.0 * lo * hi / (lo + hi) : 1.0);
    }
    for (unsigned i = 0; i < N; ++i)
        if (!std::isfinite(n_plus[i]) || !std::isfinite(n_minus[i])) return fail(c, EK_EINVAL, "ion densities must be finite");
    return EK_OK;
}

static ek_status scratch_setup(ek_ctx* c);

template <typename T>
static ek_status init_impl(ek_ctx* c, const double* rho_a, const double* rho_b, const double* n_plus,
                           const double* n_minus, const ek_particle* parts, int np) {
    const ek_params& p = c->p;
    const unsigned N = c->N;
    HostGeom g;
    EK_TRY(build_geometry(c, parts, np, g));
    const bool colloids = np > 0;
    c->S.colloids = colloids;
    EK_TRY(reference_densities(c, g, rho_a, rho_b, n_plus, n_minus));
    EK_TRY(allocate_all<T>(c, g, np));
    c->ws_mode = 0;  // later buffers come from hipMalloc
    EK_TRY(scratch_setup(c));

    const size_t es = sizeof(T);
    if (c->moment_state)
        for (int b = 0; b < 2; ++b) EK_HIP(hipMemsetAsync(c->ms[b], 0, 8 * (size_t)N * es, c->st));
    c->phi_own = c->phi;
    c->q_own = c->q;
    EK_HIP(hipHostMalloc((void**)&c->hscal, 32 * sizeof(double), hipHostMallocDefault));
    for (auto& L : c->mg) EK_HIP(hipMemsetAsync(L.phi, 0, (size_t)L.n * 8, c->st));
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 2; ++k) {
            if (c->f[b][k]) EK_HIP(hipMemsetAsync(c->f[b][k], 0, (size_t)kQ * N * es, c->st));
            EK_HIP(hipMemsetAsync(c->n[b][k], 0, (size_t)N * es, c->st));
        }
    EK_HIP(hipMemsetAsync(c->mom, 0, 8 * (size_t)N * es, c->st));
    if (c->rlo) EK_HIP(hipMemsetAsync(c->rlo, 0, 2 * (size_t)N * es, c->st));
    if (c->mlo) EK_HIP(hipMemsetAsync(c->mlo, 0, 2 * (size_t)N * es, c->st));
    EK_HIP(hipMemsetAsync(c->uph, 0, 3 * (size_t)N * es, c->st));
    EK_HIP(hipMemsetAsync(c->phi, 0, (size_t)N * 8, c->st));
    EK_HIP(hipMemsetAsync(c->scal, 0, 32 * 8, c->st));
    int hmax[16] = {0};
    hmax[8] = 1;
    EK_HIP(hipMemcpyAsync(c->obs_max, hmax, sizeof(hmax), hipMemcpyHostToDevice, c->st));
    EK_HIP(hipStreamSynchronize(c->st));  // hmax is a stack array

    // geometry upload
    c->hflags = g.flags;
    c->hpsis = g.psis;
    c->nv = (int)g.vlist.size();
    if (c->nv > 0) EK_HIP(hipMemcpyAsync(c->vlist, g.vlist.data(), g.vlist.size() * 4, hipMemcpyHostToDevice, c->st));
    c->npl = (int)g.plist.size();
    if (c->npl > 0) EK_HIP(hipMemcpyAsync(c->plist, g.plist.data(), g.plist.size() * 4, hipMemcpyHostToDevice, c->st));
    if (c->S.reproject) {
        const int32_t n0 = c->npl;
        EK_HIP(hipMemcpy(c->npl_dev, &n0, 4, hipMemcpyHostToDevice));
        const size_t B3 = (size_t)c->S.rp_box * c->S.rp_box * c->S.rp_box;
        c->npl = (int)std::max(g.plist.size(), std::min((size_t)N, (size_t)np * B3));  // launch size
    }
    if (colloids) {
        EK_HIP(hipMemcpyAsync(c->flags, g.flags.data(), N, hipMemcpyHostToDevice, c->st));
        std::vector<double> tmp(N);
        for (unsigned i = 0; i < N; ++i) tmp[i] = 1.0 - g.psis[i];
        EK_HIP(hipMemcpyAsync(c->stage, tmp.data(), (size_t)N * 8, hipMemcpyHostToDevice, c->st));
        launch_upload<T>((T*)c->psif, c->stage, N, c->st);
        EK_HIP(hipStreamSynchronize(c->st));
        EK_HIP(hipMemcpyAsync(c->stage, g.qc.data(), (size_t)N * 8, hipMemcpyHostToDevice, c->st));
        launch_upload<T>((T*)c->qc, c->stage, N, c->st);
        EK_HIP(hipMemcpyAsync(c->owner, g.owner.data(), (size_t)N * 4, hipMemcpyHostToDevice, c->st));
        EK_HIP(hipMemcpyAsync(c->linkbase, g.linkbase.data(), (size_t)N * 4, hipMemcpyHostToDevice, c->st));
        c->nlinks = g.nlinks;
        EK_HIP(hipMemsetAsync(c->linkdp, 0, (size_t)std::max(1LL, g.nlinks) * 6 * 8, c->st));
        EK_HIP(hipMemcpyAsync(c->plink_off, g.link_off.data(), g.link_off.size() * 4, hipMemcpyHostToDevice, c->st));
        EK_HIP(hipMemcpyAsync(c->plink_idx, g.link_idx.data(), g.link_idx.size() * 4, hipMemcpyHostToDevice, c->st));
        EK_HIP(hipMemcpyAsync(c->psite_off, g.site_off.data(), g.site_off.size() * 4, hipMemcpyHostToDevice, c->st));
        EK_HIP(hipMemcpyAsync(c->psite_idx, g.site_idx.data(), g.site_idx.size() * 4, hipMemcpyHostToDevice, c->st));
        // particles
        c->np = np;
        std::vector<double> hx(3 * np), hv(3 * np);
        c->hrad.resize(np);
        for (int j = 0; j < np; ++j) {
            for (int k = 0; k < 3; ++k) {
                hx[3 * j + k] = parts[j].x[k];
                hv[3 * j + k] = parts[j].v[k];
            }
            c->hrad[j] = parts[j].radius;
        }
        c->px0 = hx;
        for (int b = 0; b < 2; ++b) {
            EK_HIP(hipMemcpyAsync(c->px[b], hx.data(), 3 * np * 8, hipMemcpyHostToDevice, c->st));
            EK_HIP(hipMemcpyAsync(c->pv[b], hv.data(), 3 * np * 8, hipMemcpyHostToDevice, c->st));
        }
        EK_HIP(hipMemcpyAsync(c->prad, c->hrad.data(), np * 8, hipMemcpyHostToDevice, c->st));
        EK_HIP(hipMemsetAsync(c->pF, 0, 3 * np * 8, c->st));
        if (c->S.reproject) {
            std::vector<double> hq(np);
            for (int j = 0; j < np; ++j) hq[j] = parts[j].charge;
            EK_HIP(hipMemcpyAsync(c->pQ, hq.data(), np * 8, hipMemcpyHostToDevice, c->st));
            EK_HIP(hipStreamSynchronize(c->st));  // hq is a local vector
        }
        EK_HIP(hipStreamSynchronize(c->st));  // host staging vectors above end with this block
    }
    EK_HIP(hipStreamSynchronize(c->st));

    // initial populations and ions
    Fields<T> F = fields<T>(c);
    const double* rr[2] = {rho_a, rho_b};
    for (int s = 0; s < 2; ++s) {
        if (c->moment_state) {  // the first moments pass reads w_d rho0 from the densities themselves
            EK_HIP(hipMemcpyAsync(c->rho0 + (size_t)s * N, rr[s], (size_t)N * 8, hipMemcpyHostToDevice, c->st));
            continue;
        }
        EK_HIP(hipMemcpyAsync(c->stage, rr[s], (size_t)N * 8, hipMemcpyHostToDevice, c->st));
        launch_init_pop_flags<T>(c->S, (T*)c->f[c->cur][s], c->stage, c->S.rref[s], c->flags, c->st);
        EK_HIP(hipStreamSynchronize(c->st));
    }
    EK_HIP(hipStreamSynchronize(c->st));
    // ions: stored as mean density and ionic charge (staging holds n+ then n-)
    EK_HIP(hipMemcpyAsync(c->stage, n_plus, (size_t)N * 8, hipMemcpyHostToDevice, c->st));
    EK_HIP(hipMemcpyAsync(c->stage2, n_minus, (size_t)N * 8, hipMemcpyHostToDevice, c->st));
    launch_init_ions<T>(c->S, F, (T*)c->n[c->cur][0], (T*)c->n[c->cur][1], c->stage, c->stage2, c->st);
    EK_HIP(hipStreamSynchronize(c->st));
    EK_HIP(hipGetLastError());
    if (c->fft) {
        launch_lag_table(c->fft_tab, p.nx, p.ny, p.nz, c->st);
        if (hipfftPlan3d(&c->fft_fwd, p.nz, p.ny, p.nx, HIPFFT_D2Z) != HIPFFT_SUCCESS ||
            hipfftPlan3d(&c->fft_inv, p.nz, p.ny, p.nx, HIPFFT_Z2D) != HIPFFT_SUCCESS ||
            hipfftSetStream(c->fft_fwd, c->st) != HIPFFT_SUCCESS || hipfftSetStream(c->fft_inv, c->st) != HIPFFT_SUCCESS)
            return fail(c, EK_EHIP, "hipFFT plan creation failed");
    }
    // initial potential (with the lagged Fourier scheme too: its first step needs a solved
    // potential to lag)
    moments_pass<T>(c);
    ek_status st = poisson_solve<T>(c, p.poisson_tol, p.poisson_maxit, nullptr, nullptr);
    EK_HIP(hipMemcpyAsync(c->phi_prev, c->phi, (size_t)N * 8, hipMemcpyDeviceToDevice, c->st));
    EK_HIP(hipMemcpyAsync(c->phi_prev2, c->phi, (size_t)N * 8, hipMemcpyDeviceToDevice, c->st));
    c->ptotal = 0;
    c->rel_max = 0.0;
    if (c->fixed_cycles) EK_HIP(hipMemsetAsync(c->scal + 28, 0, 8, c->st));
    return st;
}

// Checks the parameters and sets up the context's scalars and multigrid levels: host work
// only, no device call.
static ek_status configure(ek_ctx* c, const ek_params* p, const ek_particle* parts, int32_t n_parts) {
    if (!p) return fail(c, EK_EINVAL, "null parameters");
    c->p = *p;
    if (p->nx < 2 || (p->nx & 1) || p->ny < 1 || p->nz < 1) return fail(c, EK_EINVAL, "nx must be even and >= 2; ny, nz >= 1");
    if (p->walls_z && p->nz < 3) return fail(c, EK_EINVAL, "walls need nz >= 3");
    const double Nd = (double)p->nx * p->ny * p->nz;
    if (Nd > 2147483647.0) return fail(c, EK_EINVAL, "lattice too large (more than 2^31 - 1 sites)");
    if (!(p->tau > 0.5)) return fail(c, EK_EINVAL, "tau must exceed 1/2");
    if (p->moment_state != 0 && p->moment_state != 1) return fail(c, EK_EINVAL, "moment_state must be 0 or 1");
    if (p->moment_state && (p->tau != 1.0 || n_parts > 0))
        return fail(c, EK_EINVAL, "the moment state needs tau = 1 and no particles");
    c->moment_state = p->moment_state != 0;
    c->ms_first = c->moment_state;
    if (p->precision != EK_FP32 && p->precision != EK_FP64) return fail(c, EK_EINVAL, "precision must be EK_FP32 or EK_FP64");
    if (!(p->D > 0.0) || !(p->beta > 0.0) || !(p->rho0 > 0.0)) return fail(c, EK_EINVAL, "D, beta and rho0 must be positive");
    if (!(p->eps_a > 0.0) || !(p->eps_b > 0.0) || !(p->eps_p > 0.0)) return fail(c, EK_EINVAL, "permittivities must be positive");
    if ((p->dmu[0] != 0.0 || p->dmu[1] != 0.0) && p->drho_a == 0.0) return fail(c, EK_EINVAL, "drho_a must be non-zero with solvation");
    if (n_parts < 0 || (n_parts > 0 && !parts)) return fail(c, EK_EINVAL, "bad particle array");
    for (int j = 0; j < n_parts; ++j) {
        bool ok = std::isfinite(parts[j].radius) && parts[j].radius > 0.0 && std::isfinite(parts[j].charge);
        for (int k = 0; k < 3; ++k) ok = ok && std::isfinite(parts[j].x[k]) && std::isfinite(parts[j].v[k]);
        if (!ok) return fail(c, EK_EINVAL, "particle " + std::to_string(j) + ": non-finite position, velocity or charge, or radius <= 0");
    }
    if (p->poisson_maxit < 0 || !(p->poisson_tol > 0.0)) return fail(c, EK_EINVAL, "poisson_tol must be > 0, maxit >= 0");
    if (p->phi_history < 0 || p->phi_history > 3) return fail(c, EK_EINVAL, "phi_history must be in 0..3");
    c->phi_history = p->phi_history;
    c->N = (unsigned)Nd;
    c->nblk = site_blocks(c->N);
    Scalars& S = c->S;
    S.nx = p->nx;
    S.ny = p->ny;
    S.nz = p->nz;
    S.nxy = p->nx * p->ny;
    S.N = c->N;
    S.walls = p->walls_z ? 1 : 0;
    S.kelvin = p->eps_a != p->eps_b;
    S.z0 = S.walls ? 1 : 0;
    S.z1 = S.walls ? p->nz - 2 : p->nz - 1;
    S.ndomain = (unsigned)S.nxy * (unsigned)(S.z1 - S.z0 + 1);
    // an odd periodic y or z axis (length >= 3) has no red-black colouring: three colours
    S.ncolor = ((S.ny >= 3 && (S.ny & 1)) || (!S.walls && S.nz >= 3 && (S.nz & 1))) ? 3 : 2;
    S.inv_nx = 1.0 / S.nx;
    S.inv_ny = 1.0 / S.ny;
    S.inv_nxy = 1.0 / S.nxy;
    S.inv_hx = S.nx >= 2 ? 1.0 / (S.nx / 2) : 0.0;
    if (p->reproject != 0 && p->reproject != 1) return fail(c, EK_EINVAL, "reproject must be 0 or 1");
    if (p->reproject && (n_parts == 0 || !p->move_particles))
        return fail(c, EK_EINVAL, "reproject needs particles that move (move_particles = 1)");
    S.reproject = p->reproject;
    S.subs = p->subsample > 0 ? p->subsample : 8;
    S.rp_half = S.rp_box = 0;
    if (S.reproject) {
        if (S.subs > 31) return fail(c, EK_EINVAL, "subsample must be at most 31 with reproject");
        double rmax = 0.0;
        for (int j = 0; j < n_parts; ++j) rmax = std::max(rmax, parts[j].radius);
        // a site changes only within R + 1.87 of the new centre (a move below one site, sub-cell
        // centres within sqrt(3)/2), its neighbour flags within one more; floor() of the centre
        // loses up to one more site on the low side
        S.rp_half = (int)std::ceil(rmax) + 4;
        S.rp_box = 2 * S.rp_half + 1;
        if (S.rp_box > p->nx || S.rp_box > p->ny || S.rp_box > p->nz)
            return fail(c, EK_EINVAL, "reproject needs every axis at least 2 ceil(max radius) + 9 sites long");
    }
    // banded workgroup order of the stencil sweeps (see site_banded), on request only: when
    // every z-plane is a whole number of workgroups and nz splits over the 8 XCDs
    if (p->sweep_band < -1) return fail(c, EK_EINVAL, "sweep_band must be >= -1");
    S.band = 0;
    S.plane_blocks = 0;
    S.slab_planes = 0;
    if (p->sweep_band > 0 && S.nxy % kBlock == 0 && S.nz % 8 == 0) {
        const int pb = S.nxy / kBlock;
        const int B = p->sweep_band;
        if (pb % B == 0) {
            S.band = B;
            S.plane_blocks = pb;
            S.slab_planes = S.nz / 8;
        }
    }
    S.tau = p->tau;
    S.inv_tau = 1.0 / p->tau;
    S.G = p->G;
    S.rho0 = p->rho0;
    S.D = p->D;
    S.beta = p->beta;
    const double cs2 = 1.0 / 3.0;
    S.kap_p = p->dmu[0] == 0.0 ? 0.0 : p->solvation_sign * p->beta * p->dmu[0] / (2.0 * p->drho_a);
    S.kap_m = p->dmu[1] == 0.0 ? 0.0 : p->solvation_sign * p->beta * p->dmu[1] / (2.0 * p->drho_a);
    S.G_p = p->dmu[0] == 0.0 ? 0.0 : p->solvation_sign * p->dmu[0] / (p->drho_a * cs2);
    S.G_m = p->dmu[1] == 0.0 ? 0.0 : p->solvation_sign * p->dmu[1] / (p->drho_a * cs2);
    S.ion_sc = (S.G_p != 0.0 || S.G_m != 0.0);
    if (p->polarization != 0 && p->polarization != 1) return fail(c, EK_EINVAL, "polarization must be 0 or 1");
    S.polar = p->polarization;
    S.eps_a = p->eps_a;
    S.eps_b = p->eps_b;
    S.eps_p = p->eps_p;
    S.eps_bar = 0.5 * (p->eps_a + p->eps_b);
    for (int k = 0; k < 3; ++k) {
        S.E_ext[k] = p->E_ext[k];
        S.g_body[k] = p->body_accel[k];
    }
    S.sigma0 = p->sigma_wall[0];
    S.sigma1 = p->sigma_wall[1];
    c->omega = p->sor_omega > 0.0 ? p->sor_omega : omega_for(*p);
    if (p->poisson_solver < 0 || p->poisson_solver > 3) return fail(c, EK_EINVAL, "unknown poisson_solver");
    if (p->poisson_solver == EK_POISSON_FFT && p->walls_z)
        return fail(c, EK_EINVAL, "the lagged Fourier scheme needs a periodic lattice");
    // The lagged scheme is a fixed-point iteration with one sweep per step; at the particle
    // surfaces (eps_p / eps_f = 1/8 in the paper's colloids) its error amplification exceeds
    // one and the potential diverges (on the CPU oracle as well), so it is not offered there.
    if (p->poisson_solver == EK_POISSON_FFT && p->polarization)
        return fail(c, EK_EINVAL, "the lagged Fourier scheme has no polarisation source");
    if (p->polarization && p->walls_z && p->E_ext[2] != 0.0)
        return fail(c, EK_EINVAL, "the wall faces carry no displacement: a polarising field normal to the walls is undefined");
    if (p->poisson_solver == EK_POISSON_FFT && n_parts > 0)
        return fail(c, EK_EINVAL, "the lagged Fourier scheme diverges at resolved particles; use EK_POISSON_MG or SOR");
    c->fft = p->poisson_solver == EK_POISSON_FFT;
    if (p->poisson_solver != EK_POISSON_SOR) {
        // Coarsen by two while every axis of the current level divides by 4 (so that the
        // coarse level keeps even axes for red-black ordering) and the level is large.
        int dims[3] = {p->nx, p->ny, p->nz};
        while (dims[0] % 4 == 0 && dims[1] % 4 == 0 && dims[2] % 4 == 0 && dims[0] * dims[1] * dims[2] > 512) {
            for (int k = 0; k < 3; ++k) dims[k] /= 2;
            MGLevel L{};
            L.nx = dims[0];
            L.ny = dims[1];
            L.nz = dims[2];
            L.n = (unsigned)(dims[0] * dims[1] * dims[2]);
            L.inv_nx = 1.0 / L.nx;
            L.inv_ny = 1.0 / L.ny;
            L.inv_hx = 1.0 / (L.nx / 2);
            c->mg.push_back(L);
        }
        // the coarsest grid is solved inside one workgroup's LDS (at most 4608 cells)
        if (!c->mg.empty() && c->mg.back().n > 4608) c->mg.clear();
        if (c->mg.empty() && p->poisson_solver == EK_POISSON_MG)
            return fail(c, EK_EINVAL, "multigrid needs every axis divisible by 4 and a coarsest grid of at most 4608 cells");
        if (!c->mg.empty()) {
            // SOR factor of the coarsest level (uniform-coefficient estimate).  With walls the
            // coarse grids have zero faces where z wraps, so all their nz cells form a closed
            // column, as the nz - 2 fluid layers do on the lattice: its smoothest mode sets
            // the factor.
            ek_params q = *p;
            q.nx = c->mg.back().nx;
            q.ny = c->mg.back().ny;
            q.nz = c->mg.back().nz + (p->walls_z ? 2 : 0);
            c->mg_coarse_omega = std::min(1.9, omega_for(q));
        }
    }
    if (p->poisson_cycles < 0 || p->poisson_cycles > 64) return fail(c, EK_EINVAL, "poisson_cycles must be in 0..64");
    if (p->fp32_plain_collision != 0 && p->fp32_plain_collision != 1)
        return fail(c, EK_EINVAL, "fp32_plain_collision must be 0 or 1");
    if (p->poisson_cycles > 0 && (c->mg.empty() || c->fft))
        return fail(c, EK_EINVAL, "a fixed V-cycle count needs the multigrid solver");
    c->fixed_cycles = p->poisson_cycles;
    // EK_POISSON_SITE_ORDER=1 keeps the multigrid solves in site order (a diagnostic switch:
    // the results are the same, bit for bit)
    const char* site_order = std::getenv("EK_POISSON_SITE_ORDER");
    c->split_layout = !c->mg.empty() && !(site_order && std::atoi(site_order) != 0);
    // EK_POISSON_ONE_PASS=1 runs the lattice sweeps of colour-split solves in one pass
    // (k_sor_rb) where it fits.  The results are the same, bit for bit; on gfx950 the two
    // colour passes are faster (the one-pass kernel is bound by its FP64 rows, recomputed on
    // the ring), so they are the default.
    const char* one_pass = std::getenv("EK_POISSON_ONE_PASS");
    c->one_pass = one_pass && std::atoi(one_pass) != 0;
    c->esz = p->precision == EK_FP32 ? 4 : 8;
    return EK_OK;
}

static ek_status init_dispatch(ek_ctx* c, const double* rho_a, const double* rho_b, const double* n_plus,
                               const double* n_minus, const ek_particle* parts, int32_t n_parts) {
    if (!rho_a || !rho_b || !n_plus || !n_minus) return fail(c, EK_EINVAL, "null argument");
    if (c->esz == 4) return init_impl<float>(c, rho_a, rho_b, n_plus, n_minus, parts, n_parts);
    return init_impl<double>(c, rho_a, rho_b, n_plus, n_minus, parts, n_parts);
}

extern "C" ek_status ek_init(const ek_params* p, const double* rho_a, const double* rho_b, const double* n_plus,
                             const double* n_minus, const ek_particle* parts, int32_t n_parts, void* stream,
                             ek_ctx** out) {
    if (!out) return EK_EINVAL;
    ek_ctx* c = new ek_ctx();
    *out = c;
    c->st = (hipStream_t)stream;
    EK_TRY(configure(c, p, parts, n_parts));
    return init_dispatch(c, rho_a, rho_b, n_plus, n_minus, parts, n_parts);
}

extern "C" ek_status ek_workspace_bytes(const ek_params* p, const ek_particle* parts, int32_t n_parts, size_t* bytes) {
    if (!bytes) return EK_EINVAL;
    *bytes = 0;
    ek_ctx c;
    EK_TRY(configure(&c, p, parts, n_parts));
    if (c.fft) return EK_EINVAL;  // hipFFT's plans hold a work area of their own
    HostGeom g;
    c.N = (unsigned)((size_t)p->nx * p->ny * p->nz);
    EK_TRY(build_geometry(&c, parts, n_parts, g));
    c.ws_mode = 1;
    EK_TRY(c.esz == 4 ? allocate_all<float>(&c, g, n_parts) : allocate_all<double>(&c, g, n_parts));
    *bytes = c.ws_used + 256;  // room to align an arbitrary base address
    return EK_OK;
}

extern "C" ek_status ek_init_ws(const ek_params* p, const double* rho_a, const double* rho_b, const double* n_plus,
                                const double* n_minus, const ek_particle* parts, int32_t n_parts, void* workspace,
                                size_t ws_bytes, void* stream, ek_ctx** out) {
    if (!out) return EK_EINVAL;
    ek_ctx* c = new ek_ctx();
    *out = c;
    c->st = (hipStream_t)stream;
    if (!workspace) return fail(c, EK_EINVAL, "null workspace");
    EK_TRY(configure(c, p, parts, n_parts));
    if (c->fft) return fail(c, EK_EINVAL, "the lagged Fourier scheme needs hipFFT's own work area: use ek_init");
    c->ws = (char*)workspace;
    c->ws_size = ws_bytes;
    c->ws_mode = 2;
    return init_dispatch(c, rho_a, rho_b, n_plus, n_minus, parts, n_parts);
}

extern "C" ek_status ek_step(ek_ctx* c, int32_t nsteps) {
    if (!c || !c->phi) return EK_ESTATE;
    if (c->in_batch) return fail(c, EK_ESTATE, "replica of a batch: step it with ek_batch_step");
    if (nsteps < 0) return fail(c, EK_EINVAL, "nsteps must be >= 0");
    return c->esz == 4 ? step_impl<float>(c, nsteps) : step_impl<double>(c, nsteps);
}

template <typename T>
static ek_status poisson_entry(ek_ctx* c, double tol, int maxit, int* iters, double* rel) {
    moments_pass<T>(c);
    return poisson_solve<T>(c, tol, maxit, iters, rel);
}

extern "C" ek_status ek_poisson(ek_ctx* c, double tol, int32_t maxit, int32_t* iters, double* rel_res) {
    if (!c || !c->phi) return EK_ESTATE;
    if (c->in_batch) return fail(c, EK_ESTATE, "replica of a batch: its potential is solved by ek_batch_step");
    if (!(tol > 0.0) || maxit < 0) return fail(c, EK_EINVAL, "tol must be > 0 and maxit >= 0");
    int it = 0;
    double rel = 0.0;
    ek_status s = c->esz == 4 ? poisson_entry<float>(c, tol, maxit, &it, &rel) : poisson_entry<double>(c, tol, maxit, &it, &rel);
    if (iters) *iters = it;
    if (rel_res) *rel_res = rel;
    return s;
}

template <typename T>
static ek_status observe_impl(ek_ctx* c, ek_obs* o) {
    Fields<T> F = fields<T>(c);
    launch_observe<T>(c->S, F, c->nblk, c->st);
    launch_reduce(c->red, c->nblk, 11, c->obs_max, c->scal + 8, c->st);
    EK_HIP(hipMemcpyAsync(c->hscal, c->scal, 32 * sizeof(double), hipMemcpyDeviceToHost, c->st));
    EK_HIP(hipStreamSynchronize(c->st));
    const double* v = c->hscal + 8;
    std::memset(o, 0, sizeof(*o));
    o->sum_rho[0] = v[0];
    o->sum_rho[1] = v[1];
    o->sum_n[0] = v[2];
    o->sum_n[1] = v[3];
    o->sum_q = v[4];
    o->momentum[0] = v[5];
    o->momentum[1] = v[6];
    o->momentum[2] = v[7];
    o->max_u = v[8] < 0.0 ? 0.0 : v[8];
    o->nonfinite = v[9] > 0.0;
    o->negative_ions = (int32_t)v[10];
    o->source_mean = c->last_mean;
    o->poisson_rel = c->last_rel;
    o->poisson_rel0 = c->last_rel0;
    o->poisson_rel_max = c->rel_max;
    c->rel_max = 0.0;
    if (c->fixed_cycles > 0 && c->steps > 0) {  // solves without host read-back keep their residuals on the device
        o->source_mean = c->hscal[0];
        o->poisson_rel = c->hscal[29];
        o->poisson_rel0 = c->hscal[30];
        o->poisson_rel_max = c->hscal[28];
        EK_HIP(hipMemsetAsync(c->scal + 28, 0, 8, c->st));
    }
    o->poisson_iters = c->last_iters;
    o->poisson_total = c->ptotal;
    o->poisson_mg_levels = c->mg.empty() ? 0 : (int32_t)c->mg.size() + 1;
    o->steps = c->steps;
    if (c->np > 0) {
        std::vector<double> hx(3 * c->np), hv(3 * c->np);
        EK_HIP(hipMemcpyAsync(hx.data(), c->px[c->pcur], 3 * c->np * 8, hipMemcpyDeviceToHost, c->st));
        EK_HIP(hipMemcpyAsync(hv.data(), c->pv[c->pcur], 3 * c->np * 8, hipMemcpyDeviceToHost, c->st));
        EK_HIP(hipStreamSynchronize(c->st));
        const double pi = 3.14159265358979323846;
        for (int j = 0; j < c->np; ++j) {
            const double m = c->p.particle_rho * (4.0 / 3.0) * pi * c->hrad[j] * c->hrad[j] * c->hrad[j];
            for (int k = 0; k < 3; ++k) {
                o->drift[k] += (hx[3 * j + k] - c->px0[3 * j + k]) / c->np;
                o->pmomentum[k] += m * hv[3 * j + k];
            }
        }
    }
    return o->nonfinite ? fail(c, EK_ENONFINITE, "non-finite populations or ion densities") : EK_OK;
}

// ------------------------------------------------------------------------------------
// Reverse mode: checkpointed forward run and the adjoint sweep (periodic contexts).  The
// transposed passes are FP64.  An FP32 context runs its forward steps itself; its
// checkpoints are its states widened to FP64 in an FP64 twin (c->shadow, built from the
// same parameters at each checkpointed run), whose sweep recomputes every segment in FP64
// from them and reverses it.  The gradient is then the FP64 map's, linearised along
// segments that restart from the FP32 trajectory at every checkpoint.
// ------------------------------------------------------------------------------------
static ek_status adj_check(ek_ctx* c) {
    if (!c || !c->phi) return EK_ESTATE;
    if (c->in_batch) return fail(c, EK_ESTATE, "replica of a batch: no reverse mode");
    if (c->S.walls || c->np > 0) return fail(c, EK_EINVAL, "reverse mode covers periodic lattices without particles");
    if (c->S.polar) return fail(c, EK_EINVAL, "reverse mode does not cover the polarisation source");
    if (c->moment_state) return fail(c, EK_EINVAL, "reverse mode needs stored populations (moment_state = 0)");
    if (c->fft) return fail(c, EK_EINVAL, "reverse mode differentiates a converged Poisson solve, not the lagged one");
    return EK_OK;
}

static ek_status copy_d(ek_ctx* c, void* dst, const void* src, size_t n) {
    EK_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    return EK_OK;
}

static ek_status save_ck(ek_ctx* c, int slot) {
    const size_t N = c->N;
    double* b = c->adj.ck + (size_t)slot * kCkVals * N;
    EK_TRY(copy_d(c, b, c->f[c->cur][0], kQ * N));
    EK_TRY(copy_d(c, b + kQ * N, c->f[c->cur][1], kQ * N));
    EK_TRY(copy_d(c, b + 2 * kQ * N, c->n[c->cur][0], N));
    EK_TRY(copy_d(c, b + (2 * kQ + 1) * N, c->n[c->cur][1], N));
    EK_TRY(copy_d(c, b + (2 * kQ + 2) * N, c->phi, N));
    EK_TRY(copy_d(c, b + (2 * kQ + 3) * N, c->phi_prev, N));
    EK_TRY(copy_d(c, b + (2 * kQ + 4) * N, c->phi_prev2, N));
    c->adj.ck_rate[slot] = c->rate;
    c->adj.ck_steps[slot] = c->steps;
    c->adj.ck_ptotal[slot] = c->ptotal;
    c->adj.ck_ws[2 * slot] = c->ws_order;
    c->adj.ck_ws[2 * slot + 1] = c->ws_since;
    c->adj.ck_rel0[2 * slot] = c->rel0_of[2];
    c->adj.ck_rel0[2 * slot + 1] = c->rel0_of[3];
    for (int k = 0; k < 8; ++k) c->adj.ck_kring[8 * slot + k] = c->kring[k];
    c->adj.ck_kpos[slot] = c->kpos + 8 * c->kcount;
    return EK_OK;
}

static ek_status load_ck(ek_ctx* c, int slot) {
    const size_t N = c->N;
    const double* b = c->adj.ck + (size_t)slot * kCkVals * N;
    EK_TRY(copy_d(c, c->f[c->cur][0], b, kQ * N));
    EK_TRY(copy_d(c, c->f[c->cur][1], b + kQ * N, kQ * N));
    EK_TRY(copy_d(c, c->n[c->cur][0], b + 2 * kQ * N, N));
    EK_TRY(copy_d(c, c->n[c->cur][1], b + (2 * kQ + 1) * N, N));
    EK_TRY(copy_d(c, c->phi, b + (2 * kQ + 2) * N, N));
    EK_TRY(copy_d(c, c->phi_prev, b + (2 * kQ + 3) * N, N));
    EK_TRY(copy_d(c, c->phi_prev2, b + (2 * kQ + 4) * N, N));
    c->rate = c->adj.ck_rate[slot];
    c->steps = c->adj.ck_steps[slot];
    c->ptotal = c->adj.ck_ptotal[slot];
    c->ws_order = c->adj.ck_ws[2 * slot];
    c->ws_since = c->adj.ck_ws[2 * slot + 1];
    c->rel0_of[2] = c->adj.ck_rel0[2 * slot];
    c->rel0_of[3] = c->adj.ck_rel0[2 * slot + 1];
    for (int k = 0; k < 8; ++k) c->kring[k] = c->adj.ck_kring[8 * slot + k];
    c->kpos = c->adj.ck_kpos[slot] % 8;
    c->kcount = c->adj.ck_kpos[slot] / 8;
    return EK_OK;
}

// The FP64 twin of an FP32 context, built afresh from its current parameters (the field
// included) and fields, with the same V-cycle shape.
static ek_status shadow_make(ek_ctx* c) {
    if (c->shadow) (void)ek_destroy(c->shadow);
    c->shadow = nullptr;
    const size_t N = c->N;
    std::vector<double> ra(N), rb(N), np(N), nm(N);
    EK_TRY(ek_get_field(c, EK_F_RHO_A, ra.data()));
    EK_TRY(ek_get_field(c, EK_F_RHO_B, rb.data()));
    EK_TRY(ek_get_field(c, EK_F_N_PLUS, np.data()));
    EK_TRY(ek_get_field(c, EK_F_N_MINUS, nm.data()));
    ek_params p64 = c->p;
    p64.precision = EK_FP64;
    ek_ctx* sh = nullptr;
    const ek_status st = ek_init(&p64, ra.data(), rb.data(), np.data(), nm.data(), nullptr, 0, (void*)c->st, &sh);
    if (st != EK_OK) {
        const std::string m = sh ? sh->err : std::string();
        if (sh) (void)ek_destroy(sh);
        return fail(c, st, "the FP64 twin for reverse mode: " + m);
    }
    sh->mg_fine_pre = c->mg_fine_pre;
    sh->mg_fine_post = c->mg_fine_post;
    sh->mg_pre = c->mg_pre;
    sh->mg_post = c->mg_post;
    sh->mg_tail_pre = c->mg_tail_pre;
    sh->mg_tail_post = c->mg_tail_post;
    sh->mg_coarsest = c->mg_coarsest;
    sh->mg_omega = c->mg_omega;
    c->shadow = sh;
    return EK_OK;
}

// The FP32 context's state widened into its twin: populations (deviations re-referenced to
// the twin's rho_ref, the rest population with its low part), ions, the potential and its
// two predecessors, and the host control state of the solver.
static ek_status shadow_sync(ek_ctx* c) {
    ek_ctx* sh = c->shadow;
    const unsigned N = c->N;
    for (int comp = 0; comp < 2; ++comp)
        for (int d = 0; d < kQ; ++d) {
            double* dst = (double*)sh->f[sh->cur][comp] + (size_t)d * N;
            launch_to_double<float>((const float*)c->f[c->cur][comp] + (size_t)d * N, dst, N,
                                    weight(d) * (c->S.rref[comp] - sh->S.rref[comp]), c->st);
            if (d == kRest && c->rlo) launch_add_lo<float>((const float*)c->rlo + (size_t)comp * N, dst, N, c->st);
        }
    for (int k = 0; k < 2; ++k)
        launch_to_double<float>((const float*)c->n[c->cur][k], (double*)sh->n[sh->cur][k], N, 0.0, c->st);
    EK_HIP(hipGetLastError());
    EK_TRY(copy_d(c, sh->phi, c->phi, N));
    EK_TRY(copy_d(c, sh->phi_prev, c->phi_prev, N));
    EK_TRY(copy_d(c, sh->phi_prev2, c->phi_prev2, N));
    sh->rate = c->rate;
    sh->steps = c->steps;
    sh->ptotal = c->ptotal;
    sh->ws_order = c->ws_order;
    sh->ws_since = c->ws_since;
    sh->rel0_of[2] = c->rel0_of[2];
    sh->rel0_of[3] = c->rel0_of[3];
    for (int k = 0; k < 8; ++k) sh->kring[k] = c->kring[k];
    sh->kpos = c->kpos;
    sh->kcount = c->kcount;
    return EK_OK;
}

// Room for `need` checkpoints and their host records.
static ek_status ck_alloc(ek_ctx* c, size_t need) {
    auto& A = c->adj;
    const size_t N = c->N;
    if (A.ck_cap < need) {
        dfree(c, A.ck, A.ck_cap * kCkVals * N * sizeof(double));
        A.ck = nullptr;
        A.ck_cap = 0;
        EK_TRY(dalloc(c, (void**)&A.ck, need * kCkVals * N * sizeof(double)));
        A.ck_cap = need;
    }
    A.ck_rate.assign(need, 0.0);
    A.ck_steps.assign(need, 0);
    A.ck_ptotal.assign(need, 0);
    A.ck_ws.assign(2 * need, 0);
    A.ck_rel0.assign(2 * need, 0.0);
    A.ck_kring.assign(8 * need, 0);
    A.ck_kpos.assign(need, 0);
    A.valid = false;
    return EK_OK;
}

static ek_status forward_ckpt_fp32(ek_ctx* c, int nsteps, int every) {
    const int nseg = (nsteps + every - 1) / every;
    c->adj.valid = false;
    EK_TRY(shadow_make(c));
    ek_ctx* sh = c->shadow;
    auto twin = [&](ek_status st) {  // a failure of the twin, reported on the context
        if (st != EK_OK && st != EK_ENOCONV) c->err = "FP64 twin: " + sh->err;
        return st;
    };
    EK_TRY(twin(ck_alloc(sh, (size_t)nseg + 1)));
    ek_status worst = EK_OK;
    for (int g = 0; g < nseg; ++g) {
        EK_TRY(shadow_sync(c));
        EK_TRY(twin(save_ck(sh, g)));
        const ek_status st = step_impl<float>(c, std::min(every, nsteps - g * every));
        if (st == EK_ENOCONV)
            worst = st;
        else if (st != EK_OK)
            return st;
    }
    EK_TRY(shadow_sync(c));
    EK_TRY(twin(save_ck(sh, nseg)));
    sh->adj.T = c->adj.T = nsteps;
    sh->adj.K = c->adj.K = every;
    sh->adj.nck = c->adj.nck = nseg + 1;
    sh->adj.valid = c->adj.valid = true;
    return worst;
}

extern "C" ek_status ek_forward_ckpt(ek_ctx* c, int32_t nsteps, int32_t every) {
    EK_TRY(adj_check(c));
    if (nsteps < 1 || every < 1) return fail(c, EK_EINVAL, "nsteps and every must be >= 1");
    if (c->esz == 4) return forward_ckpt_fp32(c, nsteps, every);
    auto& A = c->adj;
    const int nseg = (nsteps + every - 1) / every;
    const size_t need = (size_t)nseg + 1;
    const size_t N = c->N;
    if (A.ck_cap < need) {
        dfree(c, A.ck, A.ck_cap * kCkVals * N * sizeof(double));
        A.ck = nullptr;
        A.ck_cap = 0;
        EK_TRY(dalloc(c, (void**)&A.ck, need * kCkVals * N * sizeof(double)));
        A.ck_cap = need;
    }
    A.ck_rate.assign(need, 0.0);
    A.ck_steps.assign(need, 0);
    A.ck_ptotal.assign(need, 0);
    A.ck_ws.assign(2 * need, 0);
    A.ck_rel0.assign(2 * need, 0.0);
    A.ck_kring.assign(8 * need, 0);
    A.ck_kpos.assign(need, 0);
    A.valid = false;
    ek_status worst = EK_OK;
    for (int g = 0; g < nseg; ++g) {
        EK_TRY(save_ck(c, g));
        const ek_status st = step_impl<double>(c, std::min(every, nsteps - g * every));
        if (st == EK_ENOCONV)
            worst = st;
        else if (st != EK_OK)
            return st;
    }
    EK_TRY(save_ck(c, nseg));
    A.T = nsteps;
    A.K = every;
    A.nck = (int)need;
    A.valid = true;
    return worst;
}

extern "C" ek_status ek_adjoint(ek_ctx* c, const double* adj_f, const double* adj_n, double* grad, double* adj_f0,
                                double* adj_n0) {
    EK_TRY(adj_check(c));
    auto& A = c->adj;
    if (!A.valid) return fail(c, EK_ESTATE, "no checkpointed forward run (ek_forward_ckpt) to reverse");
    if (!adj_f || !adj_n || !grad) return fail(c, EK_EINVAL, "adj_f, adj_n and grad are required");
    if (c->esz == 4) {  // the FP64 twin holds the checkpoints and runs the sweep
        const ek_status st = ek_adjoint(c->shadow, adj_f, adj_n, grad, adj_f0, adj_n0);
        if (st != EK_OK && st != EK_ENOCONV) c->err = "FP64 twin: " + c->shadow->err;
        return st;
    }
    const size_t N = c->N;
    if (A.seg_cap < A.K) {
        dfree(c, A.seg, (size_t)A.seg_cap * kSegVals * N * sizeof(double));
        A.seg = nullptr;
        A.seg_cap = 0;
        EK_TRY(dalloc(c, (void**)&A.seg, (size_t)A.K * kSegVals * N * sizeof(double)));
        A.seg_cap = A.K;
    }
    if (!A.buf) {
        EK_TRY(dalloc(c, (void**)&A.buf, kAdjVals * N * sizeof(double)));
        EK_TRY(dalloc(c, (void**)&A.gred, (size_t)c->nblk * kRedSlots * sizeof(double)));
    }
    // adjoint field layout inside A.buf
    double* p = A.buf;
    double* lf[2][2];
    double* ln[2][2];
    for (int par = 0; par < 2; ++par)
        for (int k = 0; k < 2; ++k) {
            lf[par][k] = p;
            p += kQ * N;
        }
    for (int par = 0; par < 2; ++par)
        for (int k = 0; k < 2; ++k) {
            ln[par][k] = p;
            p += N;
        }
    AdjFields AF{};
    AF.aS = p; p += 6 * N;
    AF.aF = p; p += 3 * N;
    AF.aE = p; p += 3 * N;
    AF.arho = p; p += 2 * N;
    AF.au = p; p += 3 * N;
    AF.an = p; p += 2 * N;
    AF.aeps = p; p += N;
    AF.rhs = p; p += N;
    double* mu = p; p += N;
    double* mu1 = p; p += N;  // the adjoint potentials of the two reverse steps before
    double* mu2 = p; p += N;
    AF.mu = mu;
    AF.gred = A.gred;

    EK_HIP(hipMemsetAsync(A.gred, 0, (size_t)c->nblk * kRedSlots * sizeof(double), c->st));
    EK_HIP(hipMemsetAsync(mu, 0, 3 * N * sizeof(double), c->st));  // mu, mu1, mu2
    EK_TRY(copy_d(c, lf[0][0], adj_f, kQ * N));
    EK_TRY(copy_d(c, lf[0][1], adj_f + kQ * N, kQ * N));
    EK_TRY(copy_d(c, ln[0][0], adj_n, N));
    EK_TRY(copy_d(c, ln[0][1], adj_n + N, N));
    const double rate_fwd = c->rate;
    // The adjoint solves keep a cycle rate and cycle counts of their own, carried from one
    // reverse step to the next across segments (each recomputed segment starts from its
    // checkpoint's), so the sweep does not depend on the checkpoint interval.
    struct {
        double rate;
        int kring[8], kpos, kcount;
    } hadj = {rate_fwd, {0, 0, 0, 0, 0, 0, 0, 0}, 0, 0};
    auto swap_hist = [&]() {
        std::swap(c->rate, hadj.rate);
        for (int k = 0; k < 8; ++k) std::swap(c->kring[k], hadj.kring[k]);
        std::swap(c->kpos, hadj.kpos);
        std::swap(c->kcount, hadj.kcount);
    };
    int nadj = 0;  // adjoint solves so far
    int la = 0;
    ek_status worst = EK_OK;
    double g[kAdjSlots];
    auto sweep = [&]() -> ek_status {
        const int nseg = A.nck - 1;
        for (int g = nseg - 1; g >= 0; --g) {
            const int t0 = g * A.K, n = std::min(A.K, A.T - t0);
            // recompute the segment, keeping each step's state and the potential solved in it
            EK_TRY(load_ck(c, g));
            for (int k = 0; k < n; ++k) {
                double* b = A.seg + (size_t)k * kSegVals * N;
                EK_TRY(copy_d(c, b, c->f[c->cur][0], kQ * N));
                EK_TRY(copy_d(c, b + kQ * N, c->f[c->cur][1], kQ * N));
                EK_TRY(copy_d(c, b + 2 * kQ * N, c->n[c->cur][0], N));
                EK_TRY(copy_d(c, b + (2 * kQ + 1) * N, c->n[c->cur][1], N));
                const ek_status st = step_impl<double>(c, 1);
                if (st != EK_OK && st != EK_ENOCONV) return st;
                EK_TRY(copy_d(c, b + (2 * kQ + 2) * N, c->phi, N));
            }
            // reverse the steps of the segment
            for (int k = n - 1; k >= 0; --k) {
                double* b = A.seg + (size_t)k * kSegVals * N;
                Fields<double> F = fields<double>(c);
                F.f[0] = b;
                F.f[1] = b + kQ * N;
                F.n[0] = b + 2 * kQ * N;
                F.n[1] = b + (2 * kQ + 1) * N;
                F.phi = b + (2 * kQ + 2) * N;
                {
                    Timer tm(c, EK_T_MOMENTS);
                    launch_moments<double>(c->S, F, c->nblk, c->st);
                }
                {
                    Timer tm(c, EK_T_FORCE);
                    launch_force<double>(c->S, F, c->st);
                }
                for (int k2 = 0; k2 < 2; ++k2) {
                    AF.lf[k2] = lf[la][k2];
                    AF.lfo[k2] = lf[la ^ 1][k2];
                    AF.ln[k2] = ln[la][k2];
                    AF.lno[k2] = ln[la ^ 1][k2];
                }
                launch_adj_force(c->S, F, AF, c->st);
                launch_adj_links(c->S, F, AF, c->st);
                launch_adj_rhs(c->S, F, AF, c->st);
                launch_source_mean(c->S, c->red, c->nblk, c->scal, c->st);
                EK_HIP(hipGetLastError());
                // adjoint Poisson equation M mu = dL/dphi with the same solver: the source and
                // the unknown are swapped in for the charge and the potential.  Warm start: mu
                // varies smoothly from one reverse step to the next, so the start is extrapolated
                // in time from the solutions known so far (quadratic once there are three).
                {
                    EK_KT(EK_K_EXTRAPOLATE);
                    launch_phi_extrapolate(c->S, mu, mu1, mu2, nadj >= 3 ? 3 : (nadj >= 2 ? 2 : 1), c->st);
                }
                ++nadj;
                void* q_fwd = c->q;
                double* phi_fwd = c->phi;
                c->q = AF.rhs;
                c->phi = mu;
                c->adj_solve = true;
                swap_hist();
                const ek_status ps = poisson_solve<double>(c, c->p.poisson_tol, c->p.poisson_maxit, nullptr, nullptr);
                swap_hist();
                c->adj_solve = false;
                c->q = q_fwd;
                c->phi = phi_fwd;
                if (ps == EK_ENOCONV)
                    worst = ps;
                else if (ps != EK_OK)
                    return ps;
                launch_adj_final(c->S, F, AF, c->st);
                EK_HIP(hipGetLastError());
                la ^= 1;
            }
        }
        // parameter gradient: fixed-order sum of the per-workgroup partials
        launch_reduce(A.gred, c->nblk, kAdjSlots, nullptr, c->stage, c->st);
        EK_HIP(hipMemcpyAsync(g, c->stage, sizeof(g), hipMemcpyDeviceToHost, c->st));
        if (adj_f0) {
            EK_TRY(copy_d(c, adj_f0, lf[la][0], kQ * N));
            EK_TRY(copy_d(c, adj_f0 + kQ * N, lf[la][1], kQ * N));
        }
        if (adj_n0) {
            EK_TRY(copy_d(c, adj_n0, ln[la][0], N));
            EK_TRY(copy_d(c, adj_n0 + N, ln[la][1], N));
        }
        return EK_OK;
    };
    const ek_status sst = sweep();
    c->adj_solve = false;
    // leave the context at the end of the forward run, also after a failed sweep
    const ek_status lst = load_ck(c, A.nck - 1);
    c->rate = rate_fwd;
    if (sst != EK_OK) return sst;
    EK_TRY(lst);
    EK_HIP(hipStreamSynchronize(c->st));
    grad[0] = g[kAdjEx];
    grad[1] = g[kAdjEx + 1];
    grad[2] = g[kAdjEx + 2];
    grad[3] = g[kAdjEa] + 0.5 * g[kAdjEbar];
    grad[4] = g[kAdjEb] + 0.5 * g[kAdjEbar];
    grad[5] = g[kAdjG];
    if (worst == EK_ENOCONV) c->err = "an adjoint Poisson solve stopped at maxit above the tolerance";
    return worst;
}

// The shapes the autotuner tries, the default first.
struct CycleShape {
    int v[7];  // fine pre/post, launched coarse grids pre/post, tail grid pre/post, coarsest sweeps
    double omega;
};
static const CycleShape kCycleShapes[] = {
    {{1, 2, 1, 2, 3, 3, 10}, 1.2}, {{1, 2, 1, 2, 2, 2, 10}, 1.2}, {{1, 2, 1, 2, 4, 4, 8}, 1.2},
    {{1, 2, 1, 1, 3, 3, 10}, 1.2}, {{1, 2, 2, 2, 3, 3, 10}, 1.2}, {{1, 2, 1, 2, 3, 3, 10}, 1.3},
    {{1, 2, 1, 2, 3, 3, 20}, 1.2}, {{2, 2, 1, 2, 3, 3, 10}, 1.2},
};
constexpr int kNumCycleShapes = (int)(sizeof(kCycleShapes) / sizeof(kCycleShapes[0]));

static void apply_shape(ek_ctx* c, const CycleShape& sh) {
    c->mg_fine_pre = sh.v[0];
    c->mg_fine_post = sh.v[1];
    c->mg_pre = sh.v[2];
    c->mg_post = sh.v[3];
    c->mg_tail_pre = sh.v[4];
    c->mg_tail_post = sh.v[5];
    c->mg_coarsest = sh.v[6];
    c->mg_omega = sh.omega;
    c->rate = -1.0;        // the convergence rate of the new shape is estimated afresh
    cycles_forget(c);      // and so are the cycles a solve needs
    vcycle_graph_drop(c);  // the captured cycle has the old shape
}

extern "C" ek_status ek_set_field(ek_ctx* c, const double* E_ext) {
    if (!c || !c->phi) return EK_ESTATE;
    if (c->in_batch) return fail(c, EK_ESTATE, "replica of a batch: its field is fixed by the batch");
    if (!E_ext) return fail(c, EK_EINVAL, "null field");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(E_ext[k])) return fail(c, EK_EINVAL, "the field must be finite");
    if (c->S.polar && c->S.walls && E_ext[2] != 0.0)
        return fail(c, EK_EINVAL, "the wall faces carry no displacement: a polarising field normal to the walls is undefined");
    for (int k = 0; k < 3; ++k) c->S.E_ext[k] = c->p.E_ext[k] = E_ext[k];
    vcycle_graph_drop(c);  // the captured cycle holds the old field in its kernel arguments
    c->adj.valid = false;  // checkpoints of a run with the old field cannot be recomputed
    return EK_OK;
}

extern "C" ek_status ek_set_multigrid(ek_ctx* c, int32_t fine_pre, int32_t fine_post, int32_t coarse_pre,
                                      int32_t coarse_post, int32_t tail_pre, int32_t tail_post,
                                      int32_t coarsest_sweeps, double omega) {
    if (!c || !c->phi) return EK_ESTATE;
    if (c->in_batch) return fail(c, EK_ESTATE, "replica of a batch: its cycle is fixed by the batch");
    const int v[7] = {fine_pre, fine_post, coarse_pre, coarse_post, tail_pre, tail_post, coarsest_sweeps};
    for (int k = 0; k < 7; ++k)
        if (v[k] < 0 || v[k] > 64) return fail(c, EK_EINVAL, "sweep counts must be in 0..64");
    if (fine_pre + fine_post == 0 || coarsest_sweeps == 0)
        return fail(c, EK_EINVAL, "the lattice needs a sweep per cycle and the coarsest grid at least one");
    if (!(omega > 0.0 && omega < 2.0)) return fail(c, EK_EINVAL, "omega must be in (0, 2)");
    CycleShape sh{{fine_pre, fine_post, coarse_pre, coarse_post, tail_pre, tail_post, coarsest_sweeps}, omega};
    apply_shape(c, sh);
    return EK_OK;
}

// ------------------------------------------------------------------------------------
// Autotuner of the V-cycle shape: every candidate runs the same steps from the same saved
// state, timed with HIP events on the context's stream; the state is put back and the
// fastest shape kept.
// ------------------------------------------------------------------------------------
namespace {
struct HostState {
    int cur, pcur, ws_order, ws_since, last_iters, ms_first;
    double rate, rel0_of[4], last_rel, last_mean, last_rel0;
    long long steps, ptotal;
    int kring[8], kpos, kcount;
};
}  // namespace

// Device state copy: populations and ions of the current buffers, the three potentials,
// particle positions, velocities and last forces.
static ek_status tune_copy(ek_ctx* c, bool save, HostState& h) {
    const size_t N = c->N, pop = (size_t)kQ * N * c->esz, ion = N * c->esz, pb = (size_t)3 * c->np * 8;
    char* b = (char*)c->tune_buf;
    if (save) {
        h = HostState{c->cur, c->pcur, c->ws_order, c->ws_since, c->last_iters, c->ms_first ? 1 : 0, c->rate,
                      {0, 0, 0, 0}, c->last_rel, c->last_mean, c->last_rel0, c->steps, c->ptotal,
                      {0, 0, 0, 0, 0, 0, 0, 0}, c->kpos, c->kcount};
        for (int k = 0; k < 4; ++k) h.rel0_of[k] = c->rel0_of[k];
        for (int k = 0; k < 8; ++k) h.kring[k] = c->kring[k];
    } else {
        c->cur = h.cur;
        c->pcur = h.pcur;
        c->ws_order = h.ws_order;
        c->ws_since = h.ws_since;
        c->last_iters = h.last_iters;
        c->ms_first = h.ms_first != 0;
        c->rate = h.rate;
        for (int k = 0; k < 4; ++k) c->rel0_of[k] = h.rel0_of[k];
        c->last_rel = h.last_rel;
        c->last_mean = h.last_mean;
        c->last_rel0 = h.last_rel0;
        c->steps = h.steps;
        c->ptotal = h.ptotal;
        for (int k = 0; k < 8; ++k) c->kring[k] = h.kring[k];
        c->kpos = h.kpos;
        c->kcount = h.kcount;
    }
    // populations of the current step, or the moment state (8 N values, in the first slot)
    void* dev[] = {c->moment_state ? c->ms[c->cur] : c->f[c->cur][0], c->moment_state ? nullptr : c->f[c->cur][1],
                   c->n[c->cur][0], c->n[c->cur][1], c->phi, c->phi_prev, c->phi_prev2,
                   c->np ? c->px[c->pcur] : nullptr, c->np ? c->pv[c->pcur] : nullptr, c->np ? c->pF : nullptr, c->rlo};
    const size_t len[] = {c->moment_state ? 8 * N * c->esz : pop, pop, ion, ion, N * 8, N * 8, N * 8, pb, pb, pb,
                          c->rlo ? 2 * N * c->esz : 0};
    for (int k = 0; k < 11; ++k) {
        if (!dev[k] || !len[k]) continue;
        if (save)
            EK_HIP(hipMemcpyAsync(b, dev[k], len[k], hipMemcpyDeviceToDevice, c->st));
        else
            EK_HIP(hipMemcpyAsync(dev[k], b, len[k], hipMemcpyDeviceToDevice, c->st));
        b += (len[k] + 255) & ~(size_t)255;
    }
    return EK_OK;
}

static size_t tune_bytes(const ek_ctx* c) {
    const size_t N = c->N, pb = (size_t)3 * c->np * 8;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return 2 * up(kQ * N * c->esz) + 2 * up(N * c->esz) + 3 * up(N * 8) + 3 * up(pb) + (c->rlo ? up(2 * N * c->esz) : 0);
}

template <typename T>
static ek_status autotune_impl(ek_ctx* c, int trial, int* best, double* ms_out) {
    if (!c->tune_buf) EK_TRY(dalloc(c, &c->tune_buf, tune_bytes(c)));
    const CycleShape orig{{c->mg_fine_pre, c->mg_fine_post, c->mg_pre, c->mg_post, c->mg_tail_pre, c->mg_tail_post,
                           c->mg_coarsest},
                          c->mg_omega};
    HostState h{};
    EK_TRY(tune_copy(c, true, h));
    hipEvent_t ev[2];
    EK_HIP(hipEventCreate(&ev[0]));
    EK_HIP(hipEventCreate(&ev[1]));
    const int timing = c->timing;
    c->timing = 0;
    double per[kNumCycleShapes];
    for (int k = 0; k < kNumCycleShapes; ++k) per[k] = 1e300;
    ek_status st = EK_OK;
    // Two rounds over the candidates, each candidate's best round counts (clock and
    // thermal drift during the sweep hit every candidate alike).  Each trial: the saved
    // state, one untimed step that captures the cycle graph and estimates the cycle's
    // convergence rate, the saved state again (keeping that rate and the cycle count that
    // step recorded, so the timed steps start from this shape's own cycle floor, not the
    // one of the shape in place before the call), the timed steps.
    for (int round = 0; round < 2 && st == EK_OK; ++round)
        for (int k = 0; k < kNumCycleShapes && st == EK_OK; ++k) {
            apply_shape(c, kCycleShapes[k]);
            st = tune_copy(c, false, h);
            c->rate = -1.0;
            cycles_forget(c);
            if (st == EK_OK) st = step_impl<T>(c, 1);
            if (st == EK_ENOCONV) st = EK_OK;
            const double rate = c->rate;
            int kr[8];
            for (int j = 0; j < 8; ++j) kr[j] = c->kring[j];
            const int kp = c->kpos, kc = c->kcount;
            if (st == EK_OK) st = tune_copy(c, false, h);
            if (st != EK_OK) break;
            c->rate = rate;
            for (int j = 0; j < 8; ++j) c->kring[j] = kr[j];
            c->kpos = kp;
            c->kcount = kc;
            (void)hipEventRecord(ev[0], c->st);
            st = step_impl<T>(c, trial);
            if (st == EK_ENOCONV) st = EK_OK;
            (void)hipEventRecord(ev[1], c->st);
            if (hipEventSynchronize(ev[1]) != hipSuccess) st = EK_EHIP;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
            per[k] = std::min(per[k], (double)ms / trial);
        }
    // the fastest, unless an earlier candidate (the default first) is within 1 % of it
    int arg = 0;
    for (int k = 1; k < kNumCycleShapes; ++k)
        if (per[k] < per[arg]) arg = k;
    for (int k = 0; k < arg; ++k)
        if (per[k] <= 1.01 * per[arg]) {
            arg = k;
            break;
        }
    if (ms_out)
        for (int k = 0; k < kNumCycleShapes; ++k) ms_out[k] = per[k];
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    c->timing = timing;
    const CycleShape& b = st == EK_OK ? kCycleShapes[arg] : orig;
    apply_shape(c, b);
    const ek_status rs = tune_copy(c, false, h);
    bool same = b.omega == orig.omega;
    for (int j = 0; j < 7; ++j) same = same && b.v[j] == orig.v[j];
    if (!same) {  // the restored rate and cycle counts belong to the old shape
        c->rate = -1.0;
        cycles_forget(c);
    }
    EK_HIP(hipStreamSynchronize(c->st));
    dfree(c, c->tune_buf, tune_bytes(c));
    c->tune_buf = nullptr;
    if (st != EK_OK) return st;
    EK_TRY(rs);
    if (best) *best = arg;
    return EK_OK;
}

extern "C" int32_t ek_autotune_candidates(int32_t* shapes, double* omegas) {
    for (int k = 0; k < kNumCycleShapes; ++k) {
        if (shapes)
            for (int j = 0; j < 7; ++j) shapes[7 * k + j] = kCycleShapes[k].v[j];
        if (omegas) omegas[k] = kCycleShapes[k].omega;
    }
    return kNumCycleShapes;
}

extern "C" ek_status ek_autotune_multigrid(ek_ctx* c, int32_t trial_steps, int32_t* best, double* ms_per_step) {
    if (!c || !c->phi) return EK_ESTATE;
    if (c->in_batch) return fail(c, EK_ESTATE, "replica of a batch: its cycle is fixed by the batch");
    if (c->mg.empty()) return fail(c, EK_EINVAL, "this lattice is solved by SOR: there is no V-cycle to tune");
    if (c->fft) return fail(c, EK_EINVAL, "the lagged Fourier scheme runs no V-cycles in its steps");
    if (c->S.reproject) return fail(c, EK_EINVAL, "moving particles change the geometry, which the tuner does not restore");
    if (trial_steps < 1 || trial_steps > 1000) return fail(c, EK_EINVAL, "trial_steps must be in 1..1000");
    return c->esz == 4 ? autotune_impl<float>(c, trial_steps, best, ms_per_step)
                       : autotune_impl<double>(c, trial_steps, best, ms_per_step);
}


template <typename T>
static ek_status field_impl(ek_ctx* c, int which, double* host) {
    const unsigned N = c->N;
    Fields<T> F = fields<T>(c);
    if ((which == EK_F_PSI_S || which == EK_F_SOLID) && c->S.reproject) {  // the geometry moves: read it back
        std::vector<uint8_t> fl(N);
        std::vector<T> pf(N);
        EK_HIP(hipMemcpyAsync(fl.data(), c->flags, N, hipMemcpyDeviceToHost, c->st));
        EK_HIP(hipMemcpyAsync(pf.data(), c->psif, (size_t)N * sizeof(T), hipMemcpyDeviceToHost, c->st));
        EK_HIP(hipStreamSynchronize(c->st));
        for (unsigned i = 0; i < N; ++i) host[i] = which == EK_F_PSI_S ? 1.0 - (double)pf[i] : (double)(fl[i] & 1);
        return EK_OK;
    }
    if (which == EK_F_PSI_S || which == EK_F_SOLID) {
        for (unsigned i = 0; i < N; ++i) host[i] = which == EK_F_PSI_S ? c->hpsis[i] : (double)(c->hflags[i] & 1);
        return EK_OK;
    }
    if (which == EK_F_PHI) {
        EK_HIP(hipMemcpyAsync(host, c->phi, (size_t)N * 8, hipMemcpyDeviceToHost, c->st));
        EK_HIP(hipStreamSynchronize(c->st));
        return EK_OK;
    }
    if (which == EK_F_N_PLUS || which == EK_F_N_MINUS) {
        launch_ion_species<T>((const T*)c->n[c->cur][0], (const T*)c->n[c->cur][1], c->stage, N,
                              which == EK_F_N_PLUS ? 1.0 : -1.0, c->st);
    } else if (which >= EK_F_EX && which <= EK_F_EZ) {
        launch_field_e<T>(c->S, F, which - EK_F_EX, c->stage, c->st);
    } else {
        launch_moments<T>(c->S, F, c->nblk, c->st);
        launch_virtual<T>(c->S, F, c->st);
        const T* src = nullptr;
        double add = 0.0;
        switch (which) {
            case EK_F_RHO_A: src = (const T*)c->mom; add = c->S.rref[0]; break;
            case EK_F_RHO_B: src = (const T*)c->mom + N; add = c->S.rref[1]; break;
            case EK_F_UX: src = (const T*)c->mom + 5 * (size_t)N; break;
            case EK_F_UY: src = (const T*)c->mom + 6 * (size_t)N; break;
            case EK_F_UZ: src = (const T*)c->mom + 7 * (size_t)N; break;
            case EK_F_Q: src = (const T*)c->q; break;
            case EK_F_EPS: src = (const T*)c->eps; break;
            default: return fail(c, EK_EINVAL, "unknown field id");
        }
        launch_to_double<T>(src, c->stage, N, add, c->st);
    }
    EK_HIP(hipGetLastError());
    EK_HIP(hipMemcpyAsync(host, c->stage, (size_t)N * 8, hipMemcpyDeviceToHost, c->st));
    EK_HIP(hipStreamSynchronize(c->st));
    return EK_OK;
}

extern "C" ek_status ek_get_field(ek_ctx* c, int32_t which, double* host_out) {
    if (!c || !c->phi) return EK_ESTATE;
    if (!host_out) return fail(c, EK_EINVAL, "null output");
    if (which < 0 || which > EK_F_EZ) return fail(c, EK_EINVAL, "unknown field id");
    return c->esz == 4 ? field_impl<float>(c, which, host_out) : field_impl<double>(c, which, host_out);
}

extern "C" ek_status ek_observables(ek_ctx* c, ek_obs* out, uint32_t field_mask, double* host_fields) {
    if (!c || !c->phi) return EK_ESTATE;
    if (!out) return fail(c, EK_EINVAL, "null output");
    if (field_mask >> (EK_F_EZ + 1)) return fail(c, EK_EINVAL, "field_mask has bits beyond EK_F_EZ");
    if (field_mask && !host_fields) return fail(c, EK_EINVAL, "null host_fields with a non-zero field_mask");
    const ek_status st = c->esz == 4 ? observe_impl<float>(c, out) : observe_impl<double>(c, out);
    if (st != EK_OK && st != EK_ENONFINITE) return st;
    size_t slot = 0;
    for (int k = 0; k <= EK_F_EZ; ++k)
        if (field_mask & (1u << k)) {
            EK_TRY(c->esz == 4 ? field_impl<float>(c, k, host_fields + slot * c->N)
                               : field_impl<double>(c, k, host_fields + slot * c->N));
            ++slot;
        }
    return st;
}

// The library's observables scratch: a file-scope device array, one copy on each GPU the
// library runs on (held until the process ends).  Host code uses the address that
// hipGetSymbolAddress returns on the current device (kept per device and per context), never
// the array's name, which on the host is only a stand-in.  It holds the per-workgroup partial
// sums of ek_observables_device: at most kObsScratchBlocks workgroups x 11 values.
constexpr int kObsValues = 11;
constexpr unsigned kObsScratchBlocks = 1024;
constexpr size_t kScratchDoubles = 16384;  // 128 KiB
static_assert(kObsScratchBlocks * kObsValues <= kScratchDoubles, "observables partials exceed the scratch array");
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Once per device, with that device current: the device address of the scratch array.
static ek_status scratch_setup(ek_ctx* c) {
    int dev = 0;
    EK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, EK_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        EK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    c->obs_scratch = g_scratch_ptr[dev];
    return EK_OK;
}

template <typename T>
static ek_status observe_device_impl(ek_ctx* c, double* d_out) {
    const unsigned nblk = std::min(site_blocks(c->N), kObsScratchBlocks);
    if ((size_t)nblk * kObsValues > kScratchDoubles)
        return fail(c, EK_EINVAL, "observables partials exceed the library's scratch array");
    launch_observe_strided<T>(c->S, fields<T>(c), nblk, c->obs_scratch, c->st);
    launch_reduce(c->obs_scratch, nblk, kObsValues, c->obs_max, d_out, c->st);
    EK_HIP(hipGetLastError());
    return EK_OK;
}

extern "C" ek_status ek_observables_device(ek_ctx* c, double* d_out) {
    if (!c || !c->phi || !c->obs_scratch) return EK_ESTATE;
    if (!d_out) return fail(c, EK_EINVAL, "null output");
    return c->esz == 4 ? observe_device_impl<float>(c, d_out) : observe_device_impl<double>(c, d_out);
}

template <typename T>
static ek_status pops_impl(ek_ctx* c, int comp, double* host) {
    const unsigned N = c->N;
    if (c->moment_state) {  // gathered from the moment state into a temporary 19 N buffer
        double* buf = nullptr;
        EK_TRY(dalloc(c, (void**)&buf, (size_t)kQ * N * 8));
        launch_export_pop<T>(c->S, fields<T>(c), comp, buf, c->st);
        const hipError_t e1 = hipMemcpyAsync(host, buf, (size_t)kQ * N * 8, hipMemcpyDeviceToHost, c->st);
        const hipError_t e2 = hipStreamSynchronize(c->st);
        dfree(c, buf, (size_t)kQ * N * 8);
        EK_HIP(e1);
        EK_HIP(e2);
        return EK_OK;
    }
    for (int d = 0; d < kQ; ++d) {
        launch_to_double<T>((const T*)c->f[c->cur][comp] + (size_t)d * N, c->stage, N, weight(d) * c->S.rref[comp], c->st);
        if (d == kRest && c->rlo) launch_add_lo<T>((const T*)c->rlo + (size_t)comp * N, c->stage, N, c->st);
        EK_HIP(hipMemcpyAsync(host + (size_t)d * N, c->stage, (size_t)N * 8, hipMemcpyDeviceToHost, c->st));
        EK_HIP(hipStreamSynchronize(c->st));
    }
    return EK_OK;
}

extern "C" ek_status ek_get_populations(ek_ctx* c, int32_t comp, double* host_out) {
    if (!c || !c->phi) return EK_ESTATE;
    if (!host_out || comp < 0 || comp > 1) return fail(c, EK_EINVAL, "bad component or null output");
    return c->esz == 4 ? pops_impl<float>(c, comp, host_out) : pops_impl<double>(c, comp, host_out);
}

extern "C" ek_status ek_get_particles(ek_ctx* c, double* out) {
    if (!c || !c->phi) return EK_ESTATE;
    if (c->np == 0) return EK_OK;
    if (!out) return fail(c, EK_EINVAL, "null output");
    std::vector<double> hx(3 * c->np), hv(3 * c->np), hf(3 * c->np);
    EK_HIP(hipMemcpyAsync(hx.data(), c->px[c->pcur], 3 * c->np * 8, hipMemcpyDeviceToHost, c->st));
    EK_HIP(hipMemcpyAsync(hv.data(), c->pv[c->pcur], 3 * c->np * 8, hipMemcpyDeviceToHost, c->st));
    EK_HIP(hipMemcpyAsync(hf.data(), c->pF, 3 * c->np * 8, hipMemcpyDeviceToHost, c->st));
    EK_HIP(hipStreamSynchronize(c->st));
    for (int j = 0; j < c->np; ++j)
        for (int k = 0; k < 3; ++k) {
            out[9 * j + k] = hx[3 * j + k];
            out[9 * j + 3 + k] = hv[3 * j + k];
            out[9 * j + 6 + k] = hf[3 * j + k];
        }
    return EK_OK;
}

extern "C" ek_status ek_device_bytes(const ek_ctx* c, size_t* bytes) {
    if (!c || !bytes) return EK_EINVAL;
    *bytes = c->bytes;
    return EK_OK;
}

extern "C" ek_status ek_set_timing(ek_ctx* c, int32_t enable) {
    if (!c) return EK_EINVAL;
    resolve_timing(c);
    c->timing = enable < 0 ? 0 : (enable > 3 ? 3 : enable);
    for (int k = 0; k < EK_T_COUNT; ++k) {
        c->tms[k] = 0.0;
        c->tcnt[k] = 0;
    }
    for (int k = 0; k < EK_K_COUNT; ++k) {
        c->kms[k] = 0.0;
        c->kcnt[k] = 0;
    }
    return EK_OK;
}

extern "C" ek_status ek_get_timing(ek_ctx* c, ek_timing* out) {
    if (!c || !out) return EK_EINVAL;
    resolve_timing(c);
    for (int k = 0; k < EK_T_COUNT; ++k) {
        out->ms[k] = c->tms[k];
        out->count[k] = c->tcnt[k];
    }
    for (int k = 0; k < EK_K_COUNT; ++k) {
        out->kernel_ms[k] = c->kms[k];
        out->kernel_count[k] = c->kcnt[k];
    }
    return EK_OK;
}

extern "C" const char* ek_kernel_name(int32_t k) {
    static const char* names[EK_K_COUNT] = {
        "k_moments", "k_virtual", "k_source_mean", "k_phi_extrapolate", "k_residual", "k_reduce",
        "k_mg_coarsen", "k_sor", "k_sor_black_from", "k_mg_restrict_fine", "k_mg_restrict", "k_mg_smooth",
        "k_mg_tail", "k_mg_prolong_red_fine", "k_mg_prolong_fine", "k_mg_prolong", "k_phi_finalize", "k_force",
        "k_fused", "k_particle_step", "lagged_fourier", "k_reproject", "k_sor_rb"};
    return k >= 0 && k < EK_K_COUNT ? names[k] : "";
}

extern "C" ek_status ek_destroy(ek_ctx* c) {
    if (!c) return EK_OK;
    if (c->in_batch) return fail(c, EK_ESTATE, "replica of a batch: released by ek_batch_destroy");
    if (c->shadow) (void)ek_destroy(c->shadow);
    if (c->phi) (void)hipStreamSynchronize(c->st);
    resolve_timing(c);
    vcycle_graph_drop(c);
    if (c->fft_fwd) (void)hipfftDestroy(c->fft_fwd);
    if (c->fft_inv) (void)hipfftDestroy(c->fft_inv);
    if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
    for (auto e : c->pool) (void)hipEventDestroy(e);
    for (void* a : c->allocs) (void)hipFree(a);
    if (c->hscal) (void)hipHostFree(c->hscal);
    delete c;
    return EK_OK;
}

extern "C" const char* ek_status_str(ek_status s) {
    switch (s) {
        case EK_OK: return "ok";
        case EK_EINVAL: return "invalid argument";
        case EK_ENOMEM: return "out of memory";
        case EK_EHIP: return "HIP runtime error";
        case EK_ENOCONV: return "Poisson solve did not converge";
        case EK_ENONFINITE: return "non-finite value";
        case EK_ESTATE: return "invalid state";
        default: return "unknown status";
    }
}

extern "C" const char* ek_last_error(const ek_ctx* c) { return c ? c->err.c_str() : "null context"; }

// ------------------------------------------------------------------------------------
// Batched replicas
// ------------------------------------------------------------------------------------
struct BatchTable {
    BlockRef* d = nullptr;
    unsigned n = 0;
};

struct ek_batch {
    std::vector<ek_ctx*> reps;
    hipStream_t st = nullptr;
    std::string err;
    size_t esz = 4;
    int cycles = 4;
    int max_grid = 0;  // largest grid index over replicas
    int max_gpu = 0;   // largest grid handled by full-GPU launches
    void* desc[2] = {nullptr, nullptr};
    BatchTable site, color;
    std::vector<BatchTable> cells, cells_gpu, colors_gpu, into;  // indexed by grid
    std::vector<void*> allocs;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int parity = 0;
    long long steps = 0;
    double* hres = nullptr;
};

#define EB_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            b->err = std::string(#call) + ": " + hipGetErrorString(e_);              \
            return EK_EHIP;                                                          \
        }                                                                            \
    } while (0)

static ek_status batch_table(ek_batch* b, const std::vector<BlockRef>& h, BatchTable& t) {
    t.n = (unsigned)h.size();
    if (h.empty()) return EK_OK;
    EB_HIP(hipMalloc((void**)&t.d, h.size() * sizeof(BlockRef)));
    b->allocs.push_back(t.d);
    EB_HIP(hipMemcpy(t.d, h.data(), h.size() * sizeof(BlockRef), hipMemcpyHostToDevice));
    return EK_OK;
}

static int last_gpu_grid(const ek_ctx* c) {
    const int nl = (int)c->mg.size();
    const int tail_mid = (nl >= 2 && c->mg[nl - 2].n <= 4096 && c->mg[nl - 1].n <= 512) ? 1 : 0;
    return nl - 1 - tail_mid;
}

template <typename T>
static RepDesc<T> make_desc(ek_ctx* c, int parity) {
    const int saved = c->cur;
    c->cur = parity;
    RepDesc<T> d{};
    d.S = c->S;
    d.F = fields<T>(c);
    c->cur = saved;
    d.phi_prev = c->phi_prev;
    const int nl = (int)c->mg.size();
    d.nl = nl;
    for (int l = 0; l < nl; ++l) d.mg[l] = c->mg[l];
    d.tail_mid = (nl >= 2 && c->mg[nl - 2].n <= 4096 && c->mg[nl - 1].n <= 512) ? 1 : 0;
    d.coarse_iters = c->mg_coarsest;
    d.coarse_omega = c->mg_coarse_omega;
    d.mid_pre = c->mg_tail_pre;
    d.mid_post = c->mg_tail_post;
    d.smooth_omega = c->mg_omega;
    return d;
}

// One step of every replica, as launched (and captured) on the batch stream.
template <typename T>
static void batch_step_launches(ek_batch* b, int parity) {
    const RepDesc<T>* D = (const RepDesc<T>*)b->desc[parity];
    const int nr = (int)b->reps.size();
    hipStream_t st = b->st;
    launch_batch<T>(kB_MOMENTS, D, b->site.d, b->site.n, 0, 0, st);
    launch_batch_source_mean<T>(D, nr, st);
    launch_batch<T>(kB_EXTRAPOLATE, D, b->site.d, b->site.n, 0, 0, st);
    launch_batch<T>(kB_COARSEN_FINE, D, b->cells[1].d, b->cells[1].n, 1, 0, st);
    for (int g = 2; g <= b->max_grid; ++g) launch_batch<T>(kB_COARSEN, D, b->cells[g].d, b->cells[g].n, g, 0, st);
    for (int cyc = 0; cyc < b->cycles; ++cyc) {
        for (int g = 0; g <= b->max_gpu; ++g) {
            const int pre = g == 0 ? b->reps[0]->mg_fine_pre : b->reps[0]->mg_pre;
            for (int sweep = 0; sweep < pre; ++sweep)
                for (int color = 0; color < 2; ++color) {
                    if (g == 0)
                        launch_batch<T>(kB_SOR, D, b->color.d, b->color.n, 0, color, st);
                    else
                        launch_batch<T>(kB_SMOOTH, D, b->colors_gpu[g].d, b->colors_gpu[g].n, g, color, st);
                }
            if (g == 0)
                launch_batch<T>(kB_RESTRICT_FINE, D, b->into[1].d, b->into[1].n, 1, 0, st);
            else
                launch_batch<T>(kB_RESTRICT, D, b->into[g + 1].d, b->into[g + 1].n, g, 0, st);
        }
        launch_batch_tail<T>(D, nr, st);
        for (int g = b->max_gpu; g >= 0; --g) {
            if (g == 0)
                launch_batch<T>(kB_PROLONG_FINE, D, b->site.d, b->site.n, 0, 0, st);
            else
                launch_batch<T>(kB_PROLONG, D, b->cells_gpu[g].d, b->cells_gpu[g].n, g, 0, st);
            const int post = g == 0 ? b->reps[0]->mg_fine_post : b->reps[0]->mg_post;
            for (int sweep = 0; sweep < post; ++sweep)
                for (int color = 0; color < 2; ++color) {
                    if (g == 0)
                        launch_batch<T>(kB_SOR, D, b->color.d, b->color.n, 0, color, st);
                    else
                        launch_batch<T>(kB_SMOOTH, D, b->colors_gpu[g].d, b->colors_gpu[g].n, g, color, st);
                }
        }
    }
    launch_batch<T>(kB_RESIDUAL, D, b->site.d, b->site.n, 0, 0, st);
    launch_batch_reduce<T>(D, nr, st);
    launch_batch<T>(kB_FINALIZE, D, b->site.d, b->site.n, 0, 0, st);
    launch_batch<T>(kB_FORCE, D, b->site.d, b->site.n, 0, 0, st);
    launch_batch<T>(kB_FUSED, D, b->site.d, b->site.n, 0, 0, st);
}

// Capture one step per parity into a graph (again after a change of the cycle shape or
// count: the descriptors carry the shape and the graph the launches of each cycle).
template <typename T>
static ek_status batch_capture(ek_batch* b) {
    const int nr = (int)b->reps.size();
    EB_HIP(hipStreamSynchronize(b->st));
    for (int par = 0; par < 2; ++par) {
        std::vector<RepDesc<T>> h(nr);
        for (int r = 0; r < nr; ++r) h[r] = make_desc<T>(b->reps[r], par);
        EB_HIP(hipMemcpy(b->desc[par], h.data(), nr * sizeof(RepDesc<T>), hipMemcpyHostToDevice));
        if (b->exec[par]) (void)hipGraphExecDestroy(b->exec[par]);
        if (b->graph[par]) (void)hipGraphDestroy(b->graph[par]);
        b->exec[par] = nullptr;
        b->graph[par] = nullptr;
    }
    for (int par = 0; par < 2; ++par) {
        EB_HIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
        batch_step_launches<T>(b, par);
        EB_HIP(hipStreamEndCapture(b->st, &b->graph[par]));
        EB_HIP(hipGraphInstantiate(&b->exec[par], b->graph[par], nullptr, nullptr, 0));
    }
    return EK_OK;
}

template <typename T>
static ek_status batch_setup(ek_batch* b) {
    const int nr = (int)b->reps.size();
    // descriptors for the two buffer parities (filled by batch_capture)
    for (int par = 0; par < 2; ++par) {
        EB_HIP(hipMalloc(&b->desc[par], nr * sizeof(RepDesc<T>)));
        b->allocs.push_back(b->desc[par]);
    }
    // block tables
    auto blocks = [](unsigned n) { return (n + kBlock - 1) / kBlock; };
    std::vector<BlockRef> site, color;
    b->max_grid = 0;
    b->max_gpu = 0;
    for (int r = 0; r < nr; ++r) {
        const ek_ctx* c = b->reps[r];
        for (unsigned k = 0; k < blocks(c->N); ++k) site.push_back({r, (int)k});
        for (unsigned k = 0; k < blocks(c->N / 2); ++k) color.push_back({r, (int)k});
        b->max_grid = std::max(b->max_grid, (int)c->mg.size());
        b->max_gpu = std::max(b->max_gpu, last_gpu_grid(c));
    }
    EK_TRY(batch_table(b, site, b->site));
    EK_TRY(batch_table(b, color, b->color));
    const int G = b->max_grid + 1;
    b->cells.assign(G, BatchTable{});
    b->cells_gpu.assign(G, BatchTable{});
    b->colors_gpu.assign(G, BatchTable{});
    b->into.assign(G + 1, BatchTable{});
    for (int g = 1; g < G; ++g) {
        std::vector<BlockRef> cl, cg, cc, in;
        for (int r = 0; r < nr; ++r) {
            const ek_ctx* c = b->reps[r];
            if ((int)c->mg.size() < g) continue;
            const unsigned n = c->mg[g - 1].n;
            const int lg = last_gpu_grid(c);
            for (unsigned k = 0; k < blocks(n); ++k) cl.push_back({r, (int)k});
            if (g <= lg) {
                for (unsigned k = 0; k < blocks(n); ++k) cg.push_back({r, (int)k});
                for (unsigned k = 0; k < blocks(n / 2); ++k) cc.push_back({r, (int)k});
            }
            if (g - 1 <= lg)
                for (unsigned k = 0; k < blocks(n); ++k) in.push_back({r, (int)k});
        }
        EK_TRY(batch_table(b, cl, b->cells[g]));
        EK_TRY(batch_table(b, cg, b->cells_gpu[g]));
        EK_TRY(batch_table(b, cc, b->colors_gpu[g]));
        EK_TRY(batch_table(b, in, b->into[g]));
    }
    return batch_capture<T>(b);
}

extern "C" ek_status ek_batch_init(const ek_params* params, int32_t n_rep, const double* const* rho_a,
                                   const double* const* rho_b, const double* const* n_plus,
                                   const double* const* n_minus, int32_t cycles, ek_batch** out) {
    if (!out) return EK_EINVAL;
    ek_batch* b = new ek_batch();
    *out = b;
    if (!params || n_rep <= 0 || !rho_a || !rho_b || !n_plus || !n_minus) {
        b->err = "bad arguments";
        return EK_EINVAL;
    }
    if (cycles < 1 || cycles > 64) {
        b->err = "cycles must be in [1, 64]";
        return EK_EINVAL;
    }
    b->cycles = cycles;
    EB_HIP(hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking));
    EB_HIP(hipHostMalloc((void**)&b->hres, 2 * 8 * (size_t)n_rep, hipHostMallocDefault));
    for (int r = 0; r < n_rep; ++r) {
        const ek_params& p = params[r];
        if (p.walls_z || p.precision != params[0].precision) {
            b->err = "batched replicas are periodic and share one precision";
            return EK_EINVAL;
        }
        if (p.moment_state || p.poisson_solver == EK_POISSON_FFT) {
            b->err = "batched replicas store populations and solve with V-cycles";
            return EK_EINVAL;
        }
        ek_ctx* c = nullptr;
        ek_status s = ek_init(&p, rho_a[r], rho_b[r], n_plus[r], n_minus[r], nullptr, 0, b->st, &c);
        if (s != EK_OK) {
            b->err = "replica " + std::to_string(r) + ": " + (c ? c->err : std::string("init failed"));
            if (c) ek_destroy(c);
            return s;
        }
        b->reps.push_back(c);
        if (c->mg.empty() || (int)c->mg.size() > kMaxLevels) {
            b->err = "replica " + std::to_string(r) + ": lattice cannot be coarsened for multigrid";
            return EK_EINVAL;
        }
        c->in_batch = true;
    }
    b->esz = b->reps[0]->esz;
    EB_HIP(hipStreamSynchronize(b->st));
    return b->esz == 4 ? batch_setup<float>(b) : batch_setup<double>(b);
}

extern "C" ek_status ek_batch_step(ek_batch* b, int32_t nsteps) {
    if (!b || !b->exec[0]) return EK_ESTATE;
    for (int s = 0; s < nsteps; ++s) {
        EB_HIP(hipGraphLaunch(b->exec[b->parity], b->st));
        b->parity ^= 1;
        b->steps++;
    }
    for (ek_ctx* c : b->reps) {
        c->cur = b->parity;
        c->steps = b->steps;
    }
    return EK_OK;
}

extern "C" ek_status ek_batch_sync(ek_batch* b) {
    if (!b) return EK_EINVAL;
    EB_HIP(hipStreamSynchronize(b->st));
    return EK_OK;
}

extern "C" ek_status ek_batch_residuals(ek_batch* b, double* last, double* worst) {
    if (!b || b->reps.empty()) return EK_ESTATE;
    const int nr = (int)b->reps.size();
    for (int r = 0; r < nr; ++r) {
        EB_HIP(hipMemcpyAsync(b->hres + 2 * r, b->reps[r]->scal + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, b->st));
    }
    EB_HIP(hipStreamSynchronize(b->st));
    for (int r = 0; r < nr; ++r) {
        if (last) last[r] = b->hres[2 * r];
        if (worst) worst[r] = b->hres[2 * r + 1];
        // the running maximum restarts with each read (outside any captured graph)
        EB_HIP(hipMemsetAsync(b->reps[r]->scal + 5, 0, sizeof(double), b->st));
    }
    EB_HIP(hipStreamSynchronize(b->st));
    return EK_OK;
}

extern "C" ek_status ek_batch_replica(ek_batch* b, int32_t r, ek_ctx** ctx) {
    if (!b || !ctx || r < 0 || r >= (int)b->reps.size()) return EK_EINVAL;
    *ctx = b->reps[r];
    return EK_OK;
}

#define EK_TRY_B(x)                 \
    do {                            \
        const ek_status s_ = (x);   \
        if (s_ != EK_OK) return s_; \
    } while (0)

static ek_status batch_apply(ek_batch* b, const CycleShape& sh, int cycles) {
    for (ek_ctx* c : b->reps) apply_shape(c, sh);
    b->cycles = cycles;
    return b->esz == 4 ? batch_capture<float>(b) : batch_capture<double>(b);
}

extern "C" ek_status ek_batch_set_cycle(ek_batch* b, const int32_t* shape, double omega, int32_t cycles) {
    if (!b || !b->exec[0]) return EK_ESTATE;
    if (!shape) {
        b->err = "null shape";
        return EK_EINVAL;
    }
    for (int k = 0; k < 7; ++k)
        if (shape[k] < 0 || shape[k] > 64) {
            b->err = "sweep counts must be in 0..64";
            return EK_EINVAL;
        }
    if (shape[0] + shape[1] == 0 || shape[6] == 0 || !(omega > 0.0 && omega < 2.0) || cycles < 1 || cycles > 64) {
        b->err = "the lattice needs a sweep per cycle, the coarsest grid one; omega in (0, 2), cycles in 1..64";
        return EK_EINVAL;
    }
    CycleShape sh{{shape[0], shape[1], shape[2], shape[3], shape[4], shape[5], shape[6]}, omega};
    return batch_apply(b, sh, cycles);
}

// Autotuner of the batched launch: for every candidate V-cycle shape, the fewest V-cycles
// per step whose worst relative residual over trial_steps steps stays within max_residual,
// timed with HIP events on the batch stream from the same saved state of every replica;
// the fastest (shape, cycles) is kept and the state put back.
template <typename T>
static ek_status batch_autotune_impl(ek_batch* b, int trial, double maxres, int32_t* best, double* best_omega,
                                     double* best_ms) {
    const int nr = (int)b->reps.size();
    EB_HIP(hipStreamSynchronize(b->st));
    std::vector<HostState> hs(nr);
    for (int r = 0; r < nr; ++r) {
        ek_ctx* c = b->reps[r];
        if (!c->tune_buf && dalloc(c, &c->tune_buf, tune_bytes(c)) != EK_OK) {
            b->err = "replica " + std::to_string(r) + ": " + c->err;
            return EK_ENOMEM;
        }
        if (tune_copy(c, true, hs[r]) != EK_OK) {
            b->err = "replica " + std::to_string(r) + ": " + c->err;
            return EK_EHIP;
        }
    }
    const int par0 = b->parity;
    const long long steps0 = b->steps;
    auto restore = [&]() -> ek_status {
        for (int r = 0; r < nr; ++r)
            if (tune_copy(b->reps[r], false, hs[r]) != EK_OK) {
                b->err = "replica " + std::to_string(r) + ": " + b->reps[r]->err;
                return EK_EHIP;
            }
        b->parity = par0;
        b->steps = steps0;
        return EK_OK;
    };
    const ek_ctx* c0 = b->reps[0];
    const CycleShape was{{c0->mg_fine_pre, c0->mg_fine_post, c0->mg_pre, c0->mg_post, c0->mg_tail_pre,
                          c0->mg_tail_post, c0->mg_coarsest},
                         c0->mg_omega};
    const int was_cycles = b->cycles;
    hipEvent_t e0, e1;
    EB_HIP(hipEventCreate(&e0));
    EB_HIP(hipEventCreate(&e1));
    std::vector<double> worst(nr);
    double bms = 1e300;
    int bi = -1, bk = 0;
    ek_status st = EK_OK;
    for (int s = 0; s < kNumCycleShapes && st == EK_OK; ++s)
        for (int k = 1; k <= 8; ++k) {
            if ((st = restore()) != EK_OK || (st = batch_apply(b, kCycleShapes[s], k)) != EK_OK) break;
            if ((st = ek_batch_residuals(b, nullptr, nullptr)) != EK_OK) break;  // restarts the worst record
            (void)hipEventRecord(e0, b->st);
            if ((st = ek_batch_step(b, trial)) != EK_OK) break;
            (void)hipEventRecord(e1, b->st);
            if ((st = ek_batch_residuals(b, nullptr, worst.data())) != EK_OK) break;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double w = *std::max_element(worst.begin(), worst.end());
            if (w <= maxres) {
                // an earlier candidate within 1 % is kept (the default shape comes first)
                if (ms / trial < 0.99 * bms) {
                    bms = ms / trial;
                    bi = s;
                    bk = k;
                }
                break;  // more cycles of this shape only cost more
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == EK_OK) st = restore();
    EB_HIP(hipStreamSynchronize(b->st));  // the restoring copies read the saved state
    for (int r = 0; r < nr; ++r) {
        ek_ctx* c = b->reps[r];
        dfree(c, c->tune_buf, tune_bytes(c));
        c->tune_buf = nullptr;
    }
    if (st != EK_OK) return st;
    if (bi < 0) {  // no candidate met the bound: keep what the batch had
        EK_TRY_B(batch_apply(b, was, was_cycles));
        b->err = "no candidate met the residual bound within 8 V-cycles per step";
        return EK_ENOCONV;
    }
    EK_TRY_B(batch_apply(b, kCycleShapes[bi], bk));
    if (best) {
        for (int k = 0; k < 7; ++k) best[k] = kCycleShapes[bi].v[k];
        best[7] = bk;
    }
    if (best_omega) *best_omega = kCycleShapes[bi].omega;
    if (best_ms) *best_ms = bms;
    return EK_OK;
}

extern "C" ek_status ek_batch_autotune(ek_batch* b, int32_t trial_steps, double max_residual, int32_t* best,
                                       double* omega, double* ms_per_step) {
    if (!b || !b->exec[0]) return EK_ESTATE;
    if (trial_steps < 1 || trial_steps > 1000 || !(max_residual > 0.0)) {
        b->err = "trial_steps must be in 1..1000 and max_residual positive";
        return EK_EINVAL;
    }
    return b->esz == 4 ? batch_autotune_impl<float>(b, trial_steps, max_residual, best, omega, ms_per_step)
                       : batch_autotune_impl<double>(b, trial_steps, max_residual, best, omega, ms_per_step);
}

extern "C" ek_status ek_batch_destroy(ek_batch* b) {
    if (!b) return EK_OK;
    if (b->st) (void)hipStreamSynchronize(b->st);
    for (int par = 0; par < 2; ++par) {
        if (b->exec[par]) (void)hipGraphExecDestroy(b->exec[par]);
        if (b->graph[par]) (void)hipGraphDestroy(b->graph[par]);
    }
    for (ek_ctx* c : b->reps) {
        c->in_batch = false;
        ek_destroy(c);
    }
    for (void* a : b->allocs) (void)hipFree(a);
    if (b->hres) (void)hipHostFree(b->hres);
    if (b->st) (void)hipStreamDestroy(b->st);
    delete b;
    return EK_OK;
}

extern "C" const char* ek_batch_last_error(const ek_batch* b) { return b ? b->err.c_str() : "null batch"; }
