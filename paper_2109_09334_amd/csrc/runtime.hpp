// Host runtime types shared by the C ABI and the serving engine.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/sfft.h"
#include "kernels.hpp"

namespace sfft {

// ------------------------------------------------------------ workspace

struct Carver {
    size_t off = 0;
    template <typename X>
    X* take(char* base, size_t count) {
        off = (off + 255) & ~size_t(255);
        X* ptr = base ? reinterpret_cast<X*>(base + off) : nullptr;
        off += count * sizeof(X);
        return ptr;
    }
};

// Device buffers of one problem geometry. Complex arrays hold cx<float>
// (SFFT_MIXED) or cx<double> (SFFT_FP64); `void*` keeps one layout for both.
struct Workspace {
    char* base = nullptr;
    size_t bytes = 0;
    void* Z = nullptr;      // [nr + 1][n0][hp]  row spectra (last slot: IR residual)
    void* X = nullptr;      // [P + 2][h][n0]    column spectra (P: S, P+1: IR residual)
    void* Cl = nullptr;     // [nprod][D0][hp]   lag rows after the column inverse
    void* Dt = nullptr;     // [n0][hp]          row spectrum of D
    void* Kt = nullptr;     // [P][L0][hp]       stamp spectra along axis 1
    void* dfit = nullptr;   // [n0][n1]          IR difference image (compute type)
    double *omega, *theta, *thetaD, *lam, *cmat, *evec, *evecD;
    double *vrow, *vpart, *kap;
    double *piR, *piS, *piD;   // poly-correlation tables of R (|d| <= 2w), S and D (|d| <= w)
    double *sig0, *sig1, *pw;  // 1-D polynomial sums
    double* ped;               // pedestals c_R, c_S
    double* sky;               // smooth part of D: [max(DK,DB) + 1 + 2 w0][n1]
    double* kap1;              // its 1-D stamps: [max(DK,DB) + 1 + 2 w0][P][L1]
    double *G, *h, *L, *dsc, *rhs, *coef, *dfac, *dinv;
    int* flag;
    void** io;                 // caller buffers of the request in flight (graph replays)
    double* tsv;               // triangular solves' block results, two generations
};

inline int poly_degree(const Geom& g) { return g.dk > g.db ? g.dk : g.db; }

inline size_t carve(Workspace& w, const Geom& g, size_t cxb, size_t reb, char* base) {
    Carver c;
    const int dm = poly_degree(g);
    const int ntb = (dm + 1) * (dm + 2) / 2;
    w.Z = c.take<char>(base, cxb * (size_t)(g.nr + 1) * g.n0 * g.hp);
    w.X = c.take<char>(base, cxb * (size_t)(g.P + 2) * g.h * g.n0);
    w.Cl = c.take<char>(base, cxb * (size_t)g.nprod * g.D0 * g.hp);
    w.Dt = c.take<char>(base, cxb * (size_t)g.n0 * g.hp);
    w.Kt = c.take<char>(base, cxb * (size_t)g.P * g.L0 * g.hp);
    w.dfit = c.take<char>(base, reb * (size_t)g.n0 * g.n1);
    w.omega = c.take<double>(base, (size_t)g.npair * g.D0 * g.D1);
    w.theta = c.take<double>(base, (size_t)g.P * g.L0 * g.L1);
    w.thetaD = c.take<double>(base, (size_t)g.P * g.L0 * g.L1);
    w.lam = c.take<double>(base, (size_t)g.P * g.Q * g.L0 * g.L1);
    w.cmat = c.take<double>(base, (size_t)g.Q * g.Q);
    w.evec = c.take<double>(base, g.Q);
    w.evecD = c.take<double>(base, g.Q);
    w.vrow = c.take<double>(base, (size_t)g.n0 * (g.dk + 1) * (dm + 1) * g.D1);
    w.vpart = c.take<double>(base, polycorr_part_len(g, g.dk, dm, 2 * g.w1));
    w.kap = c.take<double>(base, (size_t)g.P * g.L0 * g.L1);
    w.piR = c.take<double>(base, (size_t)g.P * ntb * g.D0 * g.D1);
    w.piS = c.take<double>(base, (size_t)ntb * g.L0 * g.L1);
    w.piD = c.take<double>(base, (size_t)ntb * g.L0 * g.L1);
    w.sig0 = c.take<double>(base, (size_t)(g.dk + 1) * (g.dk + 1) * g.D0);
    w.sig1 = c.take<double>(base, (size_t)(g.dk + 1) * (g.dk + 1) * g.D1);
    w.pw = c.take<double>(base, 2 * (2 * dm + 1));
    w.ped = c.take<double>(base, 4);
    w.sky = c.take<double>(base, (size_t)(dm + 1 + 2 * g.w0) * g.n1);
    w.kap1 = c.take<double>(base, (size_t)(dm + 1 + 2 * g.w0) * g.P * g.L1);
    w.G = c.take<double>(base, (size_t)g.nu * g.nu);
    w.h = c.take<double>(base, g.nu);
    w.L = c.take<double>(base, (size_t)g.nu * g.nu);
    w.dsc = c.take<double>(base, g.nu);
    w.rhs = c.take<double>(base, g.nu);
    w.coef = c.take<double>(base, g.nu);
    w.dfac = c.take<double>(base, (size_t)((g.nu + 63) / 64) * 64 * 64);
    w.dinv = c.take<double>(base, (size_t)((g.nu + 63) / 64) * 2 * 64 * 64);
    w.flag = c.take<int>(base, 64);
    w.io = c.take<void*>(base, kIoSlots);
    w.tsv = c.take<double>(base, 4 * (size_t)g.nu);
    return c.off + 256;
}

// Twiddle tables of one line length.
struct Twiddles {
    void* tw = nullptr;       // n complex of the compute type: e^(-2 pi i t / n)
    void* twt = nullptr;      // pass tables of the line plan (compute type)
    double* twp = nullptr;    // 2n doubles: cos, sin of +2 pi t / n
    void* chirp = nullptr;    // Bluestein lines: the plan's chirp and bhat
    void* bhat = nullptr;     // tables (cx<double>), null otherwise
    void* twm = nullptr;      // Bluestein lines: e^(-2 pi i t / m), t < m (compute type)
};

// Per-stage HIP-event timers (enabled by sfft_profile): every stage of the
// pipeline records a start and a stop event on its stream.
struct Profiler {
    bool on = false;
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
};

struct StageTimer {
    Profiler* pr;
    const char* name;
    hipStream_t st;
    hipEvent_t a = nullptr;
    StageTimer(Profiler* p, const char* n, hipStream_t s) : pr(p), name(n), st(s) {
        if (pr && pr->on) {
            a = pr->get();
            (void)hipEventRecord(a, st);
        }
    }
    ~StageTimer() {
        if (a) {
            hipEvent_t b = pr->get();
            (void)hipEventRecord(b, st);
            pr->recs.push_back({name, a, b});
        }
    }
};

struct Plan {
    sfft_params p;
    Profiler* prof = nullptr;
    Geom g;
    LinePlan lp0, lp1;
    Twiddles t0, t1;
    Workspace ws;
    int device = 0;
    int stall_test = 0;   // triangular solves' give-up test (direct calls only)
    // Pairs the workspace holds (g.zs bytes apart): a batch of up to cap
    // same-variant requests runs as one launch per stage (gridDim.z = pairs).
    int cap = 1;
    // The whole path captured once per variant -- apply pair = fit pair or
    // not, image element type (SFFT_F32, SFFT_F64), pairs in the batch --
    // with every caller buffer read from the pair's table in its workspace;
    // a batch then costs one table write and one graph launch. The workspace
    // layout does not depend on the image type, so one workspace serves
    // both, each through its own graphs.
    hipGraphExec_t graph[2][2][kMaxBatch] = {};
    // noise decorrelation buffers (allocated on the plan's first use of it)
    char* dec = nullptr;
    size_t dec_bytes = 0;
    // serving engine: when the workspace last went idle (eviction order)
    uint64_t idle_since = 0;
};

int check_params(const sfft_params* p);
int64_t num_unknowns(const sfft_params* p);
Geom make_geom(const sfft_params* p);
// Line plan of length n (radix 16 first, then 2/4/8, 3s, then 16s) and the
// entries of its pass twiddle tables.
LinePlan make_line_plan(int n);
int pass_table_len(int n);
size_t workspace_bytes(const sfft_params* p);
int plan_run(Plan& pl, const void* rf, const void* sf, const void* r, const void* s, double* coef,
             void* d, hipStream_t st);
// The io.n (<= cap) requests of a batch, one launch per stage, through the
// plan's graph of that variant and batch size (captured on first use) or
// launched directly (graphs = false).
int plan_run_batch(Plan& pl, const IoBatch& io, bool same_pair, bool graphs, hipStream_t st);
// Status flag of pair z of the plan's last batch.
int read_pair_flag(const Plan& pl, int z, int* flag);
int flag_status(int f);
// Allocation-free path (noalloc.hip): the device address of its static
// scratch array on `device`, taken once; the whole path on that array.
int noalloc_init(int device);
int run_noalloc(int device, const sfft_params* p, const void* rf, const void* sf, const void* r,
                const void* s, double* coef, void* d, hipStream_t st);
class Engine;

}  // namespace sfft

using sfft::Plan;
using sfft::Twiddles;
using sfft::Engine;
using PlanKey = std::tuple<int, int, int, int, int, int, int, int>;

inline PlanKey key_of(const sfft_params* p) {
    return PlanKey{p->n0, p->n1, p->w0, p->w1, p->dk, p->db, p->const_phot_ratio, p->precision};
}

struct sfft_ctx {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    std::mutex mu;
    std::map<PlanKey, std::unique_ptr<Plan>> plans;       // direct-call plans
    std::map<std::pair<int, int>, Twiddles> twid;         // (n, mixed) -> tables
    int flag_host = 0;                                     // accumulated device flags
    int stall_test = 0;                                    // sfft_debug_solve_stall
    sfft::Profiler prof;
    std::unique_ptr<Engine> engine;
    char* mbuf = nullptr;                                  // crowded-mask scratch
    size_t mbuf_bytes = 0;
};


namespace sfft {
// Plan of p with the workspaces of `cap` pairs; its initialisation kernels
// run on init_stream (nullptr: the null stream, waited for).
int create_plan(sfft_ctx* ctx, const sfft_params* p, std::unique_ptr<Plan>& out, int cap,
                hipStream_t init_stream = nullptr);
void destroy_plan(sfft_ctx* ctx, std::unique_ptr<Plan>& pl);
}  // namespace sfft
