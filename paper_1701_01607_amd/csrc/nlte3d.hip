// nlte3d.hip -- host runtime and C-ABI of the MI355X non-LTE library.
//
// One translation unit: the kernels (kernels.h) and their constant tables live here.
// A job owns a grid hierarchy (level 0 = coarsest) with device-resident primitives,
// local-physics constants, populations and right-hand sides.  The drivers below follow
// the MALI iteration, the FAS V-cycle and full multigrid of Bjorgen & Leenaarts (2017),
// Sect. 2.1-2.3, with the conventions stated in include/nlte3d.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/nlte3d.h"
#include "kernels.h"

#include <cstdarg>
#include <fstream>
#include <sstream>

using namespace nlte;

namespace {

struct Error : std::runtime_error {
    nlte_status code;
    Error(nlte_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            throw Error(NLTE_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define REQUIRE(cond, msg) \
    do {                   \
        if (!(cond)) throw Error(NLTE_E_INVALID, msg); \
    } while (0)

inline unsigned blocks_for(size_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

// True for memory the device can address directly (device or managed allocations), so that
// entry points whose kernels take caller pointers reject host memory instead of faulting.
inline bool device_memory(const void* p) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();   // host memory unknown to the runtime: clear the error
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

}  // namespace

// ===================================================================== scratch
// Device scratch of the allocation-free entry point (nlte_emergent_intensity_noalloc):
// the emergent-intensity plane state of one frequency chunk.  Each GPU the library runs
// on holds its own copy until the process ends.  In host code `scratch` is only a
// stand-in symbol: its device address comes from hipGetSymbolAddress, per device, once.
constexpr size_t kScratchBytes = size_t(48) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (current), looked up on the first call per device.
hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

// ===================================================================== context
struct nlte_ctx {
    std::map<std::string, int> tile_cache;   // autotuned sweep tile per level shape
    std::mutex tune_mu;
    std::string tune_path;   // NLTE3D_TUNE_CACHE: autotune results kept on disk across processes
    std::string arch;        // device architecture, part of the on-disk keys
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    std::atomic<size_t> used{0};             // bytes allocated by this context
    std::atomic<size_t> reserved{0};         // bytes reserved for admitted served jobs
    std::string err;
    std::recursive_mutex mu;                 // API calls and the job map
    std::map<int64_t, struct JobBase*> jobs;
    int64_t next_job = 1;
    // serving: FIFO admission by HBM footprint, one worker thread per running job
    std::mutex qmu;
    std::condition_variable qcv;
    std::deque<struct JobBase*> queue;       // lock order: mu before qmu; workers take qmu only
    std::vector<std::thread> workers;
    int max_running = 0, running = 0;
    int batch_max = 1;                       // served jobs one worker may run as one batch
    int next_batch = 1;                      // ids of serving batches
    bool stopping = false;
    void* scratch = nullptr;                 // this device's `scratch` (device address)
};

// Autotune cache file: one flat JSON object {"<arch>|<level key>": <directions per block>, ...}.
// Unreadable or malformed files count as empty; entries with other values are skipped.
static std::map<std::string, int> read_tune_file(const std::string& path) {
    std::map<std::string, int> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t i = t.find('{');
    if (i == std::string::npos) return m;
    for (;;) {
        const size_t q0 = t.find('"', i + 1);
        if (q0 == std::string::npos) break;
        const size_t q1 = t.find('"', q0 + 1);
        const size_t colon = q1 == std::string::npos ? q1 : t.find(':', q1 + 1);
        if (colon == std::string::npos) return {};
        char* end = nullptr;
        const long v = std::strtol(t.c_str() + colon + 1, &end, 10);
        if (end == t.c_str() + colon + 1) return {};
        if (v == 3 || v == 6 || v == 12) m[t.substr(q0 + 1, q1 - q0 - 1)] = int(v);
        i = size_t(end - t.c_str());
    }
    return m;
}

static void write_tune_file(const std::string& path, const std::map<std::string, int>& m) {
    const std::string tmp = path + ".tmp" + std::to_string(reinterpret_cast<uintptr_t>(&m));
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{";
        bool first = true;
        for (const auto& kv : m) {
            f << (first ? "\n  \"" : ",\n  \"") << kv.first << "\": " << kv.second;
            first = false;
        }
        f << "\n}\n";
        if (!f) return;
    }
    std::rename(tmp.c_str(), path.c_str());
}


namespace {

// Progress lines on stderr when NLTE3D_LOG is set (long solves: one line per finest-level
// smoothing pass and per cycle, printed after the work has finished on the device).
bool log_enabled() {
    static const bool on = std::getenv("NLTE3D_LOG") != nullptr;
    return on;
}
void log_line(const char* fmt, ...) {
    std::va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "[nlte3d] ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    std::fflush(stderr);
    va_end(ap);
}

// Device buffer accounted against the context budget.
struct DevBuf {
    nlte_ctx* ctx = nullptr;
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    // `reserved`: the bytes were already reserved at admission (served jobs)
    void alloc(nlte_ctx* c, size_t b, bool reserved = false) {
        release();
        ctx = c;
        if (b == 0) return;
        if (!reserved && c->used + c->reserved + b > c->budget)
            throw Error(NLTE_E_OOM, "HBM budget exceeded: need " + std::to_string(b) + " more bytes, " +
                                        std::to_string(c->budget - c->used - c->reserved) + " left");
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error(NLTE_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
        bytes = b;
        c->used += b;
    }
    void release() {
        if (p) {
            (void)hipFree(p);
            ctx->used -= bytes;
        }
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ----------------------------------------------------------------- constant tables
// Table of the small-damping FP32 Voigt evaluation: G = 1 - 2uF(u) (F Dawson's function)
// on intervals of width 1/16 in u, as the cubic Hermite interpolant of G and
// G' = -2F - 2uG between the nodes, in monomial form in the local coordinate s in [0, 1).
// F at the nodes comes from fourth-order Runge-Kutta integration of F' = 1 - 2uF, F(0) = 0,
// with 64 steps per interval (the equation is stable forward; error ~1e-14).
void dawson_table(std::vector<float4>& tab) {
    const int sub = 64;
    const double h = 1.0 / kDawInvStep, dt = h / sub;
    auto rhs = [](double u, double F) { return 1.0 - 2.0 * u * F; };
    std::vector<double> F(kDawIntervals + 1, 0.0);
    double f = 0.0, u = 0.0;
    for (int i = 0; i < kDawIntervals; ++i) {
        for (int j = 0; j < sub; ++j) {
            const double k1 = rhs(u, f), k2 = rhs(u + 0.5 * dt, f + 0.5 * dt * k1);
            const double k3 = rhs(u + 0.5 * dt, f + 0.5 * dt * k2), k4 = rhs(u + dt, f + dt * k3);
            f += dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
            u = (i * sub + j + 1) * dt;
        }
        F[i + 1] = f;
    }
    tab.resize(kDawIntervals);
    for (int i = 0; i < kDawIntervals; ++i) {
        const double u0 = i * h, u1 = (i + 1) * h;
        const double G0 = 1.0 - 2.0 * u0 * F[i], G1 = 1.0 - 2.0 * u1 * F[i + 1];
        const double D0 = h * (-2.0 * F[i] - 2.0 * u0 * G0), D1 = h * (-2.0 * F[i + 1] - 2.0 * u1 * G1);
        tab[i] = make_float4(float(G0), float(D0), float(3.0 * (G1 - G0) - 2.0 * D0 - D1),
                             float(2.0 * (G0 - G1) + D0 + D1));
    }
}

// A4 set: per octant the permutations of (1/3, 1/3, sqrt(7)/3); 12 upward directions
// (x and y signs over the 4 upper octants), then the 12 reflections through the origin.
void a4_set(double* mu) {
    const double m1 = 1.0 / 3.0, m2 = std::sqrt(1.0 - 2.0 * m1 * m1);
    const double base[3][3] = {{m1, m1, m2}, {m1, m2, m1}, {m2, m1, m1}};
    const double sg[4][2] = {{1, 1}, {1, -1}, {-1, 1}, {-1, -1}};
    int d = 0;
    for (int o = 0; o < 4; ++o)
        for (int b = 0; b < 3; ++b, ++d) {
            mu[3 * d] = sg[o][0] * base[b][0];
            mu[3 * d + 1] = sg[o][1] * base[b][1];
            mu[3 * d + 2] = base[b][2];
        }
    for (int e = 0; e < 12; ++e)
        for (int c = 0; c < 3; ++c) mu[3 * (12 + e) + c] = -mu[3 * e + c];
}

void upload_constants() {
    std::vector<float4> dg;
    dawson_table(dg);
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_dawg), dg.data(), sizeof(float4) * kDawIntervals));
    double mu[kNDir * 3];
    a4_set(mu);
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_mu), mu, sizeof(mu)));
}

}  // namespace

// ===================================================================== atom / atmos
struct nlte_atom {
    AtomInfo info{};
    std::vector<double> q;        // flat velocity offsets, atom line order
    std::vector<double> wnu;      // flat trapezoid weights in Hz
    std::vector<int> line_of;
    int nf = 0;
    // active continua: frequencies, 2 h nu^3/c^2, and per continuum [ncont][nfc] the
    // cross-sections (0 below the edge) and 4 pi w / (h nu) with w the trapezoid weights
    // over the grid points at or above the edge
    std::vector<double> cnu, ce, calpha, cfw;
};

struct nlte_atmos {
    int nx = 0, ny = 0, nz = 0, nline_chic = 0;
    double dx = 0, dy = 0;
    std::vector<double> z;
    DevBuf prim;                  // [7 + nline_chic][nvox]
};

// ===================================================================== job
struct JobBase {
    virtual ~JobBase() = default;
    // serving state (jobs created by nlte_submit)
    bool served = false;
    std::atomic<int> state{2};       // 0 queued, 1 running, 2 done, 3 failed
    nlte_status final_status = NLTE_OK;
    std::string error;
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t footprint = 0;
    int batch_id = 0;                   // serving batch the job ran in (0: alone)
    const nlte_atmos* src_atmos = nullptr;
    const nlte_atom* src_atom = nullptr;
    hipStream_t own_stream = nullptr;
    hipStream_t batch_stream = nullptr;   // set while the job runs in a batch: all its work goes there
    virtual void build_served() = 0;
    nlte_params params{};
    int N = 0, nline = 0, nf = 0, nlev = 1, prec = NLTE_FP64;
    std::vector<double> history;
    nlte_result res{};
    virtual void run(nlte_result* out) = 0;
    virtual void formal_solution_out(int level, void* jeff, void* oml, int mem) = 0;
    virtual double mali_hook(int level, int iters) = 0;
    virtual double rate_solve_hook(int level, const void* jeff, const void* oml, int mem) = 0;
    virtual void residual_out(int level, double* dst, int mem) = 0;
    virtual void vcycle_hook(int level, int first) = 0;
    virtual long long repair_count() = 0;
    virtual void stats(nlte_result* out) = 0;
    virtual void get_pops(int level, double* dst, int mem) = 0;
    virtual void set_pops(int level, const double* src, int mem) = 0;
    virtual void source_function(double* dst, int mem) = 0;
    virtual void emergent(int ndir, const double* mu, float* dst, int mem) = 0;
    virtual void emergent_into(int ndir, const double* mu, float* dst, double* state, size_t state_bytes) = 0;
    virtual void emergent_continuum(int ndir, const double* mu, float* dst, int mem) = 0;
    virtual void restrict_hook(int level, int nq, const double* src, double* dst) = 0;
    virtual void prolong_hook(int level, int nq, const double* src, double* dst) = 0;
};

namespace {

struct Level {
    int nx = 0, ny = 0, nz = 0;
    size_t nxy = 0, nvox = 0;
    double dx = 0, dy = 0;
    std::vector<double> z;
    DevBuf dz, prim, sc, sv, nstar, pfix, ntot, n, f, nb, tmp, acc, lc, partial;
    DevBuf cr, chkT, cF, cacc;   // active continua: LTE ratios, h/kT, spontaneous rates, sums
    bool fs_valid = false;
    long long fs_count = 0;
    int nslot = 2;   // direction-group slots in acc written by the last formal solution
    int fc = 1;      // frequency chunks per (direction, tile): fixed by the level shape
    int maxslot = 8; // direction-group slots allocated in acc (8 allows every block shape)
};

// Frequency chunks per (direction, tile) wave group of the plane-step sweep.  With one
// wave per (direction, 64 plane points, line) a launch on a small plane holds less than
// two rounds of a full GPU (six waves per SIMD on 1024 SIMDs), and its last round runs
// partly empty (64x64: 7680 waves, a second round a quarter full); splitting each line's
// frequencies over 2 or 4 waves evens the rounds out.  FP32 only (the FP64 kernel's
// registers allow one).
constexpr double kSweepWaveTarget = 2.0 * 6.0 * 1024.0;
inline double sweep_waves(size_t nxy, int nline) { return double((nxy + 63) / 64) * nline * kNDir; }
inline int freq_chunks_for(size_t nxy, int nline, size_t rbytes) {
    if (rbytes != 4) return 1;
    int fc = 1;
    while (fc < 4 && sweep_waves(nxy, nline) * fc < kSweepWaveTarget) fc *= 2;
    return fc;
}

// Directions per block of the work-list sweep for a level with fc frequency chunks: FP32
// blocks hold 12 waves (12/fc directions), FP64 blocks three directions (their registers
// allow one wave per SIMD).
inline int list_block_dirs(size_t rbytes, int fc) { return rbytes == 8 ? 3 : kMaxSweepWaves / fc; }

// Accumulator slots for a level: 8, which allow every block shape down to three
// directions per block, wherever the 8-slot accumulators take at most 48 GiB (in FP32 with
// five lines up to ~160 M voxels), else 2 (12-direction blocks).  Small blocks pay on
// large planes too: on 504x504 planes three-direction blocks re-read fewer upwind cells
// from HBM than twelve-direction ones (the autotuner picks them there).
inline int acc_slots(size_t nvox, int nline, size_t rbytes) {
    return double(2 * kMaxSlots) * nline * double(nvox) * double(rbytes) <= 48.0 * 1073741824.0 ? kMaxSlots : 2;
}

template <typename R>
struct Job : JobBase {
    nlte_ctx* ctx;
    std::vector<std::unique_ptr<Level>> lev;
    DevBuf atom_d, qf, wf, line_of_d, state, topI, scalar, repairs, estate, eout, flag, nprev;
    // active continua: frequency tables (R for the sweep, FP64 for the setup) and plane state
    DevBuf ctab_r, cnu_d, ce_d, cfw_d, calpha_d, cstate, cestate;
    int nfc = 0;
    AtomInfo info{};
    int DB = 0;   // directions per sweep block (0: autotuned per level)
    int nstate = 2;   // plane-state slots: the plane being swept and its upwind plane
    int fine_db = 0;   // block shape of the last finest-level formal solution
    std::vector<double> hz_top;
    double updates_per_fs_fine = 0;
    double cost_units = 0;
    double updates = 0;
    long long sweep_launches = 0;
    double ms_setup = 0;

    // phase timing with HIP events on the context stream (params.timing)
    enum { EV_SWEEP = 0, EV_RATES = 1, EV_TRANSFER = 2 };
    struct Ev { hipEvent_t a, b; int kind; };
    std::vector<Ev> evs;
    double ms_phase[3] = {0, 0, 0};

    // Active continua: their sweep needs only the populations, so outside graph capture it
    // runs on a stream of its own, forked from the job's stream at the start of each formal
    // solution and joined before the rate equations read its sums.
    hipStream_t cstream = nullptr;
    hipEvent_t cfork = nullptr, cjoin = nullptr;

    Job(nlte_ctx* c) : ctx(c) {}
    ~Job() override {
        if (cstream) {
            (void)hipStreamSynchronize(cstream);
            (void)hipStreamDestroy(cstream);
        }
        if (cfork) (void)hipEventDestroy(cfork);
        if (cjoin) (void)hipEventDestroy(cjoin);
        for (auto& e : evs) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (own_stream) {
            (void)hipStreamSynchronize(own_stream);
            lev.clear();
            (void)hipStreamDestroy(own_stream);
        }
    }

    bool capturing = false;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<long long> graph_fs;
    double graph_cost = 0, graph_updates = 0;
    long long graph_launches = 0;

    void ev_begin(int kind) {
        if (!params.timing || capturing) return;
        Ev e;
        e.kind = kind;
        HIPCHK(hipEventCreate(&e.a));
        HIPCHK(hipEventCreate(&e.b));
        HIPCHK(hipEventRecord(e.a, st()));
        evs.push_back(e);
    }
    void ev_end() {
        if (!params.timing || capturing) return;
        HIPCHK(hipEventRecord(evs.back().b, st()));
    }
    void ev_resolve() {
        if (evs.empty()) return;
        HIPCHK(hipStreamSynchronize(st()));
        for (auto& e : evs) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
            ms_phase[e.kind] += ms;
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        evs.clear();
    }

    hipStream_t st() const { return batch_stream ? batch_stream : own_stream ? own_stream : ctx->stream; }

    // all device buffers of a job come through here
    void dalloc(DevBuf& b, size_t bytes) { b.alloc(ctx, bytes, served); }

    void build_served() override { build(src_atmos, src_atom, &params); }

    // --------------------------------------------------------------- setup
    void build(const nlte_atmos* atm, const nlte_atom* atom, const nlte_params* p) {
        auto tb = std::chrono::steady_clock::now();
        params = *p;
        info = atom->info;
        N = info.N;
        nline = info.nline;
        nf = atom->nf;
        nlev = std::max(1, p->method == NLTE_MALI ? 1 : p->nlev);
        REQUIRE(nlev <= kMaxLevels, "nlev too large");
        REQUIRE(atm->nline_chic == 0 || atm->nline_chic >= nline, "chi_c has fewer lines than the atom");
        const int step = 1 << (nlev - 1);
        REQUIRE(atm->nx % step == 0 && atm->ny % step == 0 && (atm->nz - 1) % step == 0,
                "grid " + std::to_string(atm->nx) + "x" + std::to_string(atm->ny) + "x" + std::to_string(atm->nz) +
                    " does not admit " + std::to_string(nlev) + " grid levels (need nx, ny, nz-1 divisible by " +
                    std::to_string(step) + ")");
        REQUIRE(nlev == 1 || atm->nz >= 3, "multigrid needs nz >= 3");
        if (herm())
            REQUIRE(p->sweep_kernel == NLTE_SWEEP_AUTO || p->sweep_kernel == NLTE_SWEEP_PLANE_STEP,
                    "Hermite upwind interpolation runs in the plane-step sweep only");
        if (p->method != NLTE_MALI) REQUIRE(nlev >= 1, "nlev >= 1");

        dalloc(atom_d, sizeof(AtomInfo));
        HIPCHK(hipMemcpyAsync(atom_d.p, &info, sizeof(AtomInfo), hipMemcpyHostToDevice, st()));
        std::vector<R> qh(atom->q.begin(), atom->q.end()), wh(atom->wnu.begin(), atom->wnu.end());
        dalloc(qf, sizeof(R) * nf);
        dalloc(wf, sizeof(R) * nf);
        dalloc(line_of_d, sizeof(int) * nf);
        HIPCHK(hipMemcpyAsync(qf.p, qh.data(), sizeof(R) * nf, hipMemcpyHostToDevice, st()));
        HIPCHK(hipMemcpyAsync(wf.p, wh.data(), sizeof(R) * nf, hipMemcpyHostToDevice, st()));
        if (info.cont_active) {
            nfc = int(atom->cnu.size());
            auto up = [&](DevBuf& bd, const std::vector<double>& h) {
                dalloc(bd, sizeof(double) * h.size());
                HIPCHK(hipMemcpyAsync(bd.p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st()));
            };
            up(cnu_d, atom->cnu);
            up(ce_d, atom->ce);
            up(cfw_d, atom->cfw);
            up(calpha_d, atom->calpha);
            // the sweep's per-frequency rows in precision R
            std::vector<R> tab(size_t(nfc) * kContRow, R(0));
            for (int k = 0; k < nfc; ++k) {
                R* row = tab.data() + size_t(k) * kContRow;
                row[0] = R(atom->cnu[k]);
                row[1] = R(atom->ce[k]);
                for (int t = 0; t < info.ncont; ++t) {
                    row[2 + t] = R(atom->calpha[size_t(t) * nfc + k]);
                    row[2 + kMaxCont + t] = R(atom->cfw[size_t(t) * nfc + k]);
                }
            }
            dalloc(ctab_r, sizeof(R) * tab.size());
            HIPCHK(hipMemcpyAsync(ctab_r.p, tab.data(), sizeof(R) * tab.size(), hipMemcpyHostToDevice, st()));
            HIPCHK(hipStreamSynchronize(st()));   // tab is a host temporary
        }
        HIPCHK(hipMemcpyAsync(line_of_d.p, atom->line_of.data(), sizeof(int) * nf, hipMemcpyHostToDevice, st()));
        dalloc(scalar, sizeof(double) * 4);
        dalloc(repairs, sizeof(unsigned long long));
        dalloc(flag, sizeof(int));
        HIPCHK(hipMemsetAsync(repairs.p, 0, sizeof(unsigned long long), st()));

        const int nprim = 7 + atm->nline_chic;
        maxfreq = 0;
        for (int l = 0; l < nline; ++l) maxfreq = std::max(maxfreq, info.line[l].nfreq);
        lev.resize(nlev);
        for (int k = nlev - 1; k >= 0; --k) {
            lev[k].reset(new Level());
            Level& L = *lev[k];
            if (k == nlev - 1) {
                L.nx = atm->nx; L.ny = atm->ny; L.nz = atm->nz; L.dx = atm->dx; L.dy = atm->dy; L.z = atm->z;
            } else {
                const Level& F = *lev[k + 1];
                L.nx = F.nx / 2; L.ny = F.ny / 2; L.nz = (F.nz - 1) / 2 + 1;
                L.dx = 2 * F.dx; L.dy = 2 * F.dy;
                for (int i = 0; i < F.nz; i += 2) L.z.push_back(F.z[i]);
            }
            L.nxy = size_t(L.nx) * L.ny;
            L.nvox = L.nxy * L.nz;
            L.fc = herm() ? 1 : freq_chunks(L);
            dalloc(L.dz, sizeof(double) * L.nz);
            HIPCHK(hipMemcpyAsync(L.dz.p, L.z.data(), sizeof(double) * L.nz, hipMemcpyHostToDevice, st()));
            dalloc(L.prim, sizeof(double) * nprim * L.nvox);
            if (k == nlev - 1) {
                HIPCHK(hipMemcpyAsync(L.prim.p, atm->prim.p, sizeof(double) * nprim * L.nvox,
                                      hipMemcpyDeviceToDevice, st()));
            } else {
                const Level& F = *lev[k + 1];
                restrict_kernel<<<blocks_for(L.nvox * nprim, 256), 256, 0, st()>>>(
                    F.prim.as<double>(), L.prim.as<double>(), nprim, F.nx, F.ny, F.nz, p->coarse_atmos);
                HIPCHK(hipGetLastError());
            }
            dalloc(L.sc, sizeof(R) * SC_NQ * nline * L.nvox);
            dalloc(L.sv, sizeof(R) * SV_NQ * L.nvox);
            dalloc(L.nstar, sizeof(double) * N * L.nvox);
            dalloc(L.pfix, sizeof(double) * N * N * L.nvox);
            dalloc(L.ntot, sizeof(double) * L.nvox);
            dalloc(L.n, sizeof(double) * N * L.nvox);
            dalloc(L.f, sizeof(double) * N * L.nvox);
            dalloc(L.nb, sizeof(double) * N * L.nvox);
            dalloc(L.tmp, sizeof(double) * N * L.nvox);
            L.maxslot = acc_slots(L.nvox, nline, sizeof(R));
            if (herm())
                REQUIRE(L.maxslot >= kMaxSlots, "Hermite upwind interpolation needs 8 accumulator slots per "
                                                "quantity (at most 48 GiB of them per level)");
            dalloc(L.acc, sizeof(R) * 2 * size_t(L.maxslot) * nline * L.nvox);
            dalloc(L.lc, sizeof(R) * 2 * nline * L.nvox);
            dalloc(L.partial, sizeof(double) * std::max<size_t>(blocks_for(L.nvox, 256), 1024));
            SetupArgs<R> sa;
            sa.atom = atom_d.as<AtomInfo>();
            sa.prim = L.prim.as<double>();
            sa.has_chic = atm->nline_chic ? 1 : 0;
            sa.nvox = L.nvox;
            sa.sc = L.sc.as<R>();
            sa.sv = L.sv.as<R>();
            sa.nstar = L.nstar.as<double>();
            sa.pfix = L.pfix.as<double>();
            sa.ntot = L.ntot.as<double>();
            setup_level_kernel<R><<<blocks_for(L.nvox, 128), 128, 0, st()>>>(sa);
            HIPCHK(hipGetLastError());
            profile_norm_kernel<R><<<blocks_for(L.nvox, 128), 128, 0, st()>>>(
                atom_d.as<AtomInfo>(), qf.as<R>(), wf.as<R>(), L.sc.as<R>(), L.sv.as<R>(), L.nvox);
            HIPCHK(hipGetLastError());
            fine_rhs_kernel<<<blocks_for(L.nvox, 256), 256, 0, st()>>>(L.f.as<double>(), L.ntot.as<double>(), N, L.nvox);
            HIPCHK(hipGetLastError());
            if (info.cont_active) {
                const int nct = info.ncont;
                dalloc(L.cr, sizeof(R) * nct * L.nvox);
                dalloc(L.chkT, sizeof(R) * L.nvox);
                dalloc(L.cF, sizeof(double) * nct * L.nvox);
                dalloc(L.cacc, sizeof(R) * (2 + info.cont_nup) * nct * kMaxSlots * L.nvox);
                cont_setup_kernel<R><<<blocks_for(L.nvox, 128), 128, 0, st()>>>(
                    atom_d.as<AtomInfo>(), L.prim.as<double>(), L.nstar.as<double>(), cnu_d.as<double>(),
                    ce_d.as<double>(), cfw_d.as<double>(), calpha_d.as<double>(), nfc, L.cr.as<R>(), L.chkT.as<R>(),
                    L.cF.as<double>(), L.nvox);
                HIPCHK(hipGetLastError());
            }
        }
        if (info.cont_active) {
            const Level& Fc = *lev[nlev - 1];
            // a direction's column of continuum cells is addressed by 32-bit buffer offsets
            REQUIRE(double(sizeof(CCell<R>)) * double(nfc) * double(Fc.nxy) <= 4294967295.0,
                    "continuum frequency grid too large for this plane size");
            dalloc(cstate, sizeof(CCell<R>) * 2 * kNDir * size_t(nfc) * Fc.nxy);
        }
        const Level& Fz = *lev[nlev - 1];
        // Frequency passes: each pass sweeps Q frequencies of every line.  One pass is the
        // default; the plane state (2 x 24 x nline x Q cells per plane point) is split into
        // more passes only when a single pass would take more than a quarter of the
        // context's HBM budget (NLTE3D_SWEEP_STATE_MB overrides the state size cap).
        const char* envb = std::getenv("NLTE3D_SWEEP_STATE_MB");
        const double cap_bytes = envb ? std::atof(envb) * 1048576.0 : 0.25 * double(ctx->budget);
        // a pass's (direction, line) column is addressed by 32-bit buffer offsets
        const double colmax = 4294967295.0 / (double(sizeof(Cell<R>)) * double(Fz.nxy));
        const double per_q = double(sizeof(Cell<R>)) * nstate * kNDir * nline * Fz.nxy;
        Qpass = std::max(1, std::min(maxfreq, int(cap_bytes / per_q)));
        Qpass = std::max(1, std::min(Qpass, int(colmax)));
        // planes shrink towards the coarse levels, so the finest level sizes the plane state
        dalloc(state, sizeof(Cell<R>) * nstate * kNDir * size_t(nline) * Qpass * Fz.nxy);
        dalloc(nprev, sizeof(double) * N * Fz.nvox);
        if (p->top_I) {
            dalloc(topI, sizeof(R) * size_t(nf) * Fz.nxy);
            std::vector<R> th(size_t(nf) * Fz.nxy);
            for (size_t i = 0; i < th.size(); ++i) th[i] = R(p->top_I[i]);
            HIPCHK(hipMemcpyAsync(topI.p, th.data(), sizeof(R) * th.size(), hipMemcpyHostToDevice, st()));
            HIPCHK(hipStreamSynchronize(st()));
        }
        updates_per_fs_fine = double(Fz.nvox) * kNDir * nf;

        // initial populations
        const int k0 = (p->method == NLTE_FMG) ? 0 : nlev - 1;
        Level& L0 = *lev[k0];
        if (p->init == NLTE_INIT_USER) {
            REQUIRE(p->init_pops != nullptr, "init_pops is NULL");
            REQUIRE(p->method != NLTE_FMG, "user initial populations are for MALI/FAS");
            HIPCHK(hipMemcpyAsync(L0.n.p, p->init_pops, sizeof(double) * N * L0.nvox, hipMemcpyHostToDevice, st()));
        } else if (p->init == NLTE_INIT_LTE) {
            HIPCHK(hipMemcpyAsync(L0.n.p, L0.nstar.p, sizeof(double) * N * L0.nvox, hipMemcpyDeviceToDevice, st()));
        } else {
            zero_radiation(k0);
        }
        HIPCHK(hipStreamSynchronize(st()));
        if (log_enabled())
            for (int k = 0; k < nlev; ++k) {
                const Level& L = *lev[k];
                log_line("level %d (%dx%dx%d): plane-step sweep, %d frequency chunks per wave group", k, L.nx,
                         L.ny, L.nz, L.fc);
            }
        choose_tile();
        ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
    }

    void choose_tile() {
        const int t = params.dirs_per_block;
        DB = (t == 3 || t == 6 || t == 12) ? t : 0;
    }

    std::vector<int> level_tile;   // autotuned directions per block, per level
    int maxfreq = 0, Qpass = 1;    // frequencies per line swept per pass

    std::string tile_key(const Level& L) const {
        return std::to_string(sizeof(R)) + ":" + std::to_string(L.nx) + "x" + std::to_string(L.ny) + "x" +
               std::to_string(L.nz) + ":" + std::to_string(nline) + ":" + std::to_string(nf);
    }

    static dim3 sweep_grid(const Level& L, int nline, int db) {
        return dim3(blocks_for(L.nxy, 64), nline, kNDir / db);
    }

    // Frequency chunks per wave group of this level (freq_chunks_for).
    int freq_chunks(const Level& L) const { return freq_chunks_for(L.nxy, nline, sizeof(R)); }

    bool herm() const { return params.sc_interp == NLTE_SC_HERMITE; }

    void launch_step(const SweepArgs<R>& a, dim3 grid, int db, int fc, int s) {
        const unsigned threads = unsigned(db * fc * 64);
        if (herm()) {
            sweep_step_kernel<R, 3, true><<<grid, 3 * 64, 0, st()>>>(a, s);
            return;
        }
        switch (db) {
            case 12: sweep_step_kernel<R, 12><<<grid, threads, 0, st()>>>(a, s); break;
            case 6: sweep_step_kernel<R, 6><<<grid, threads, 0, st()>>>(a, s); break;
            default: sweep_step_kernel<R, 3><<<grid, threads, 0, st()>>>(a, s); break;
        }
    }

    // Autotuner: time plane steps 1..3 of a formal solution for each block shape and keep
    // the fastest.  Every shape sums the directions by the same tree, so the choice does
    // not change results.  It is cached per (precision, shape, lines, frequencies) in the
    // context, so a shape is tuned once per process.
    int autotune_tile(int k, SweepArgs<R>& a) {
        Level& L = *lev[k];
        const std::string key = tile_key(L);
        {
            std::lock_guard<std::mutex> lk(ctx->tune_mu);
            auto it = ctx->tile_cache.find(key);
            if (it != ctx->tile_cache.end()) return it->second;
        }
        const int cand[3] = {12, 6, 3};
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        // three rounds, candidate order rotated each round, plane steps 1..6 timed
        float total[3] = {0.f, 0.f, 0.f};
        const int steps = std::min(L.nz, 7);
        for (int round = 0; round < 3; ++round) {
            for (int q = 0; q < 3; ++q) {
                const int i = (q + round) % 3;
                const int c = cand[i];
                if (c * L.fc > kMaxSweepWaves || kNDir / c > L.maxslot) continue;
                const dim3 grid = sweep_grid(L, nline, c);
                launch_step(a, grid, c, L.fc, 0);
                HIPCHK(hipEventRecord(e0, st()));
                for (int s = 1; s < steps; ++s) launch_step(a, grid, c, L.fc, s);
                HIPCHK(hipEventRecord(e1, st()));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                total[i] += ms;
            }
        }
        int best = L.maxslot >= kMaxSlots ? 3 : 12;
        float best_ms = 1e30f;
        for (int i = 0; i < 3; ++i) {
            if (cand[i] * L.fc > kMaxSweepWaves || kNDir / cand[i] > L.maxslot) continue;
            if (total[i] < best_ms) { best_ms = total[i]; best = cand[i]; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        auto it = ctx->tile_cache.find(key);
        if (it != ctx->tile_cache.end()) return it->second;   // another job tuned it first
        ctx->tile_cache[key] = best;
        if (!ctx->tune_path.empty()) {   // merge into the file (other devices' entries kept)
            auto m = read_tune_file(ctx->tune_path);
            m[ctx->arch + "|" + key] = best;
            write_tune_file(ctx->tune_path, m);
        }
        return best;
    }

    int tile_for(int k, SweepArgs<R>& a) {
        if (herm()) return 3;
        if (DB && DB * lev[k]->fc <= kMaxSweepWaves && kNDir / DB <= lev[k]->maxslot) return DB;
        if (level_tile.size() != size_t(nlev)) level_tile.assign(nlev, 0);
        if (!level_tile[k]) {
            a.m0 = 0;
            a.Q = Qpass;
            a.add = 0;
            level_tile[k] = autotune_tile(k, a);
        }
        return level_tile[k];
    }

    // --------------------------------------------------------------- kernels
    // `given`: acc holds two slots per quantity written by rate_solve_hook, whatever the
    // level's sweep layout
    void rate_launch(int k, int mode, const double* base, double* out, double sign, bool want_C,
                     bool given = false) {
        Level& L = *lev[k];
        RateArgs<R> ra;
        ra.atom = atom_d.as<AtomInfo>();
        ra.nvox = L.nvox;
        ra.pfix = L.pfix.as<double>();
        ra.acc = L.acc.as<R>();
        ra.nslot = given ? 2 : L.nslot;
        ra.n = L.n.as<double>();
        ra.f = L.f.as<double>();
        ra.base = base;
        ra.out = out;
        ra.sign = sign;
        ra.mode = mode;
        const unsigned nb = blocks_for(L.nvox, 256);
        ra.partial = want_C ? L.partial.as<double>() : nullptr;
        ra.cacc = info.cont_active ? L.cacc.as<R>() : nullptr;
        ra.cF = info.cont_active ? L.cF.as<double>() : nullptr;
        ev_begin(EV_RATES);
        switch (N) {
#define RCASE(NN) case NN: rate_kernel<R, NN><<<nb, 256, 0, st()>>>(ra); break;
            RCASE(2) RCASE(3) RCASE(4) RCASE(5) RCASE(6) RCASE(7) RCASE(8)
#undef RCASE
            default: throw Error(NLTE_E_INVALID, "number of levels must be 2..8");
        }
        HIPCHK(hipGetLastError());
        if (want_C) {
            reduce_max_kernel<<<1, 256, 0, st()>>>(L.partial.as<double>(), int(nb), scalar.as<double>());
            HIPCHK(hipGetLastError());
        }
        ev_end();
    }

    void zero_radiation(int k) {
        rate_launch(k, 1, nullptr, nullptr, 0.0, false);
        lev[k]->fs_valid = false;
    }

    // Line coefficients k+, e of level k from its populations (Sect. 3).
    void line_coef(int k) {
        Level& L = *lev[k];
        line_coef_kernel<R><<<blocks_for(L.nvox, 256), 256, 0, st()>>>(atom_d.as<AtomInfo>(), L.n.as<double>(),
                                                                      L.lc.as<R>(), L.nvox);
        HIPCHK(hipGetLastError());
    }

    // Arguments of level k's plane-step sweep (frequency pass fields left to the caller).
    SweepArgs<R> sweep_args(int k) {
        Level& L = *lev[k];
        SweepArgs<R> a{};
        a.atom = atom_d.as<AtomInfo>();
        a.nx = L.nx; a.ny = L.ny; a.nz = L.nz; a.nf = nf;
        a.nxy = unsigned(L.nxy); a.nvox = L.nvox;
        a.dx = L.dx; a.dy = L.dy;
        a.z = L.dz.as<double>();
        a.sc = L.sc.as<R>(); a.sv = L.sv.as<R>(); a.lc = L.lc.as<R>();
        a.qf = qf.as<R>(); a.wf = wf.as<R>();
        a.topI = (k == nlev - 1 && topI.p) ? topI.as<R>() : nullptr;
        a.state = state.as<Cell<R>>();
        a.acc = L.acc.as<R>();
        a.nstate = nstate;
        a.fc = L.fc;
        return a;
    }

    // Bookkeeping after a formal solution of level k.
    void fs_account(int k) {
        Level& L = *lev[k];
        L.fs_valid = true;
        ++L.fs_count;
        const Level& F = *lev[nlev - 1];
        cost_units += double(L.nvox) / double(F.nvox);
        updates += double(L.nvox) * kNDir * (nf + nfc);
    }

    // True where level k can share work-list sweep launches with other jobs: the plane-step
    // sweep with bilinear upwind interpolation, one frequency pass, no active continua, and
    // accumulator slots for the work list's block shape.
    bool list_sweep_ok(int k) const {
        const Level& L = *lev[k];
        return !herm() && Qpass >= maxfreq && !info.cont_active && !capturing &&
               kNDir / list_block_dirs(sizeof(R), L.fc) <= L.maxslot;
    }

    // The job's part of a work-list formal solution of level k: its line coefficients and
    // sweep arguments (all frequencies in one pass, overwrite the sums).
    SweepArgs<R> list_prepare(int k) {
        line_coef(k);
        SweepArgs<R> a = sweep_args(k);
        a.m0 = 0;
        a.Q = Qpass;
        a.add = 0;
        return a;
    }

    // After the shared launches: db directions per block wrote kNDir/db slots per quantity.
    void list_finish(int k, int db, long long launches) {
        lev[k]->nslot = kNDir / db;
        if (k == nlev - 1) fine_db = db;
        sweep_launches += launches;
        fs_account(k);
    }

    void formal_solution(int k) {
        Level& L = *lev[k];
        const bool cont_forked = info.cont_active && !capturing;
        if (cont_forked) cont_fork(k);
        line_coef(k);
        SweepArgs<R> a = sweep_args(k);
        const int db = tile_for(k, a);
        if (k == nlev - 1) fine_db = db;
        const dim3 grid = sweep_grid(L, nline, db);
        ev_begin(EV_SWEEP);
        for (int m0 = 0; m0 < maxfreq; m0 += Qpass) {
            a.m0 = m0;
            a.Q = Qpass;
            a.add = m0 > 0 ? 1 : 0;
            for (int s = 0; s < L.nz; ++s) launch_step(a, grid, db, L.fc, s);
            sweep_launches += L.nz;
        }
        HIPCHK(hipGetLastError());
        ev_end();
        L.nslot = kNDir / db;
        if (info.cont_active) {
            if (cont_forked) {
                ev_begin(EV_SWEEP);   // the part of the continuum sweep not hidden by the lines
                HIPCHK(hipStreamWaitEvent(st(), cjoin, 0));
                ev_end();
            } else {
                cont_sweep(k, st());
            }
        }
        fs_account(k);
    }

    // Formal solution at the continuum frequencies of level k (active continua), enqueued on
    // `stream` (the job's stream, or the continuum stream between fork and join).
    void cont_sweep(int k, hipStream_t stream) {
        Level& L = *lev[k];
        ContArgs<R> c;
        c.atom = atom_d.as<AtomInfo>();
        c.nx = L.nx; c.ny = L.ny; c.nz = L.nz; c.nfc = nfc;
        c.nxy = unsigned(L.nxy); c.nvox = L.nvox;
        c.dx = L.dx; c.dy = L.dy;
        c.z = L.dz.as<double>();
        c.n = L.n.as<double>();
        c.cr = L.cr.as<R>(); c.hkT = L.chkT.as<R>();
        c.ctab = ctab_r.as<R>();
        c.state = cstate.as<CCell<R>>();
        c.acc = L.cacc.as<R>();
        const dim3 grid(blocks_for(L.nxy, 64), 1, kNDir / 3);
        // frequency chunks: as for the line sweep, until a launch holds two rounds of waves
        int fc = 1;
        while (fc < cont_max_chunks<R>() && sweep_waves(L.nxy, 1) * fc < kSweepWaveTarget) fc *= 2;
        const bool own = stream == st();
        if (own) ev_begin(EV_SWEEP);
        const dim3 block(unsigned(3 * fc * 64));
        for (int s = 0; s < L.nz; ++s) {
            switch (info.cont_nup) {
                case 1: sweep_cont_kernel<R, 1><<<grid, block, 0, stream>>>(c, s); break;
                case 2: sweep_cont_kernel<R, 2><<<grid, block, 0, stream>>>(c, s); break;
                case 3: sweep_cont_kernel<R, 3><<<grid, block, 0, stream>>>(c, s); break;
                case 4: sweep_cont_kernel<R, 4><<<grid, block, 0, stream>>>(c, s); break;
                default: throw Error(NLTE_E_INVALID, "continuum upper-level count out of range");
            }
        }
        HIPCHK(hipGetLastError());
        if (own) ev_end();
    }

    // Starts level k's continuum sweep on the continuum stream after everything enqueued so
    // far on the job's stream (the populations it reads are final for this formal solution).
    void cont_fork(int k) {
        if (!cstream) {
            HIPCHK(hipStreamCreateWithFlags(&cstream, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&cfork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&cjoin, hipEventDisableTiming));
        }
        HIPCHK(hipEventRecord(cfork, st()));
        HIPCHK(hipStreamWaitEvent(cstream, cfork, 0));
        cont_sweep(k, cstream);
        HIPCHK(hipEventRecord(cjoin, cstream));
    }

    double read_scalar() {
        double c = 0;
        HIPCHK(hipMemcpyAsync(&c, scalar.p, sizeof(double), hipMemcpyDeviceToHost, st()));
        HIPCHK(hipStreamSynchronize(st()));
        return c;
    }

    // `iters` MALI iterations; the accumulators are reused for the first one if valid.
    void mali(int k, int iters) {
        Level& L = *lev[k];
        for (int it = 0; it < iters; ++it) {
            if (!(it == 0 && L.fs_valid)) formal_solution(k);
            rate_launch(k, 0, nullptr, nullptr, 0.0, true);
            L.fs_valid = false;
        }
        if (log_enabled() && !capturing && k == nlev - 1 && iters > 0) {
            HIPCHK(hipStreamSynchronize(st()));
            log_line("level %d (%dx%dx%d): %d MALI iterations done", k, L.nx, L.ny, L.nz, iters);
        }
    }

    // out = base + sign * W(n) with W at the current accumulators of level k.
    void apply_W(int k, const double* base, double* out, double sign) {
        rate_launch(k, 2, base, out, sign, false);
    }

    void restrict_fields(int kf, int nq, const double* src, double* dst) {
        const Level& F = *lev[kf];
        const Level& C = *lev[kf - 1];
        ev_begin(EV_TRANSFER);
        restrict_kernel<<<blocks_for(C.nvox * nq, 256), 256, 0, st()>>>(src, dst, nq, F.nx, F.ny, F.nz,
                                                                          params.restriction);
        HIPCHK(hipGetLastError());
        ev_end();
    }

    void prolong_fields(int kf, int nq, const double* src, double* dst) {
        const Level& F = *lev[kf];
        prolong_kernel<<<blocks_for(F.nvox * nq, 256), 256, 0, st()>>>(src, dst, nq, F.nx, F.ny, F.nz,
                                                                      F.dz.as<double>(), params.interpolation);
        HIPCHK(hipGetLastError());
    }

    // One FAS V-cycle on levels k..0 (Sect. 2.2).
    void vcycle(int k, bool first) {
        Level& L = *lev[k];
        const int nu_pre = (first && params.nu0 > 0) ? params.nu0 : params.nu1;
        if (k == 0) {
            mali(k, nu_pre);
            mali(k, params.nu2);
            return;
        }
        mali(k, nu_pre);
        if (!L.fs_valid) formal_solution(k);                // the extra formal solution (Eq. 7)
        vc_restrict(k);
        formal_solution(k - 1);                             // W*(R n), shared with the first coarse iteration
        vc_coarse_rhs(k);
        if (k - 1 == 0) mali(0, params.nu3);
        else vcycle(k - 1, false);
        vc_correct(k);
        mali(k, params.nu2);
    }

    // V-cycle phases between the formal solutions and smoothing passes (Sect. 2.2).
    // Residual r = f - W(n) at the accumulators of level k (Eq. 7); restriction of n and r.
    void vc_restrict(int k) {
        Level& L = *lev[k];
        apply_W(k, L.f.as<double>(), L.tmp.as<double>(), -1.0);
        L.fs_valid = false;
        Level& C = *lev[k - 1];
        restrict_fields(k, N, L.n.as<double>(), C.n.as<double>());
        restrict_fields(k, N, L.tmp.as<double>(), C.tmp.as<double>());
    }

    // Coarse right-hand side f = R r + W(R n) from the coarse accumulators (Eq. 10), and
    // n_before = R n kept for the relative correction.
    void vc_coarse_rhs(int k) {
        Level& C = *lev[k - 1];
        apply_W(k - 1, C.tmp.as<double>(), C.f.as<double>(), 1.0);
        dcopy(C.n.as<double>(), C.nb.as<double>(), size_t(N) * C.nvox);
    }

    // Relative correction interpolated to level k with the negative-population repair
    // (Eqs. 11-12, Sect. 4.10).
    void vc_correct(int k) {
        Level& L = *lev[k];
        Level& C = *lev[k - 1];
        if (params.interpolation == NLTE_INTERP_HERMITE) {
            // e on the coarse grid first (C.tmp is free once the coarse right-hand side is formed)
            const size_t nc = size_t(N) * C.nvox;
            rel_correction_kernel<<<blocks_for(nc, 256), 256, 0, st()>>>(C.n.as<double>(), C.nb.as<double>(),
                                                                          C.tmp.as<double>(), nc);
            HIPCHK(hipGetLastError());
        }
        correct_kernel<<<blocks_for(L.nvox * N, 256), 256, 0, st()>>>(
            L.n.as<double>(), C.n.as<double>(), C.nb.as<double>(), N, L.nx, L.ny, L.nz, L.dz.as<double>(),
            params.repair_frac, repairs.as<unsigned long long>(), C.tmp.as<double>(), params.interpolation);
        HIPCHK(hipGetLastError());
        L.fs_valid = false;
    }

    void cycle_change_enqueue(int k) {
        Level& L = *lev[k];
        const size_t n = size_t(N) * L.nvox;
        const unsigned nb = std::min<unsigned>(blocks_for(n, 256), 1024);
        rel_change_kernel<<<nb, 256, 0, st()>>>(L.n.as<double>(), nprev.as<double>(), n, L.partial.as<double>());
        reduce_max_kernel<<<1, 256, 0, st()>>>(L.partial.as<double>(), int(nb), scalar.as<double>());
        HIPCHK(hipGetLastError());
    }

    double cycle_change(int k) {
        cycle_change_enqueue(k);
        return read_scalar();
    }

    void dcopy(const double* src, double* dst, size_t n) {
        copy_kernel<<<std::min<unsigned>(blocks_for(n, 256), 2048), 256, 0, st()>>>(src, dst, n);
        HIPCHK(hipGetLastError());
    }

    // Capture `work` once into a HIP graph on the job's private stream, then launch the
    // graph (the captured work must be the same every time it is called).
    template <typename F>
    void replay(F&& work) {
        if (!own_stream) {
            HIPCHK(hipStreamSynchronize(ctx->stream));
            HIPCHK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
        }
        if (!gexec) {
            std::vector<long long> fs0(lev.size());
            for (size_t k = 0; k < lev.size(); ++k) fs0[k] = lev[k]->fs_count;
            const double c0 = cost_units, u0 = updates;
            const long long l0 = sweep_launches;
            capturing = true;
            HIPCHK(hipStreamBeginCapture(own_stream, hipStreamCaptureModeThreadLocal));
            try {
                work();
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(own_stream, &g);
                if (g) (void)hipGraphDestroy(g);
                capturing = false;
                throw;
            }
            HIPCHK(hipStreamEndCapture(own_stream, &graph));
            capturing = false;
            HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
            // the capture ran the host side once; record its bookkeeping as per-launch deltas
            graph_fs.assign(lev.size(), 0);
            for (size_t k = 0; k < lev.size(); ++k) {
                graph_fs[k] = lev[k]->fs_count - fs0[k];
                lev[k]->fs_count = fs0[k];
            }
            graph_cost = cost_units - c0;
            graph_updates = updates - u0;
            graph_launches = sweep_launches - l0;
            cost_units = c0;
            updates = u0;
            sweep_launches = l0;
        }
        HIPCHK(hipGraphLaunch(gexec, own_stream));
        // bookkeeping the captured work did on the host (formal-solution counts) repeats
        for (size_t k = 0; k < lev.size(); ++k) lev[k]->fs_count += graph_fs[k];
        cost_units += graph_cost;
        updates += graph_updates;
        sweep_launches += graph_launches;
    }

    // Stop rule (Eq. 18): E = rho/(1-rho) C, rho = C_i/C_{i-1}, valid in the asymptotic
    // linear regime; the first correction (from the initial populations) is excluded, so
    // rho needs the second and a later correction of the sequence h.
    bool stop(const std::vector<double>& h, double& rho, double& E) {
        const double C = h.back();
        rho = h.size() >= 3 ? C / h[h.size() - 2] : INFINITY;
        E = (rho < 1.0) ? rho / (1.0 - rho) * C : INFINITY;
        if (params.tol_C > 0 && C <= params.tol_C) return true;
        if (params.E_target > 0 && rho < 1.0 && E <= params.E_target) return true;
        return false;
    }

    // Divergence guard of the cycles (Sect. 4.10): a non-finite correction, or C growing
    // (C_i > diverge_growth C_{i-1} with C_i above 1e-3, where a converging run no longer
    // is) in diverge_cycles consecutive cycles.  `run` counts the growing cycles so far.
    const char* diverging(int& run) const {
        const double C = history.back();
        if (!std::isfinite(C)) return "non-finite cycle correction";
        const int K = params.diverge_cycles == 0 ? 3 : params.diverge_cycles;
        if (K < 0 || history.size() < 2) return nullptr;
        const double g = params.diverge_growth > 0 ? params.diverge_growth : 1.0;
        run = (C > g * history[history.size() - 2] && C > 1e-3) ? run + 1 : 0;
        return run >= K ? "growing cycle correction" : nullptr;
    }

    void check_finite(int k) {
        Level& L = *lev[k];
        HIPCHK(hipMemsetAsync(flag.p, 0, sizeof(int), st()));
        finite_check_kernel<<<blocks_for(size_t(N) * L.nvox, 256), 256, 0, st()>>>(L.n.as<double>(),
                                                                                   size_t(N) * L.nvox, flag.as<int>());
        int h = 0;
        HIPCHK(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, st()));
        HIPCHK(hipStreamSynchronize(st()));
        if (h) throw Error(NLTE_E_DIVERGED, "non-finite populations");
    }

    // Progress of one run (nlte_job_run, or a batch in which the job takes part).
    struct RunState {
        std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
        int status = NLTE_W_NOT_CONVERGED;
        int iters = 0, cycles = 0, grow_run = 0, fell_back = 0;
        double rho = INFINITY, E = INFINITY;
        bool first = true;   // the next cycle is the run's first (nu0)
    };

    int max_iterations() const { return params.max_iter > 0 ? params.max_iter : 1000; }

    bool is_mali() const {
        return params.method == NLTE_MALI || (nlev == 1 && params.method != NLTE_FAS && params.method != NLTE_FMG);
    }

    // Full multigrid from the coarsest grid (Sect. 2.3): nu_FMG iterations there, then per
    // finer grid the interpolated full approximation (Eq. 14) and one V-cycle below the top.
    void fmg_prologue() {
        mali(0, params.nu_fmg);
        for (int k = 1; k <= nlev - 1; ++k) fmg_lift(k);
    }
    void fmg_lift(int k) {
        prolong_fields(k, N, lev[k - 1]->n.as<double>(), lev[k]->n.as<double>());
        lev[k]->fs_valid = false;
        if (k < nlev - 1) vcycle(k, false);
    }

    // After a MALI iteration whose C is in history: true when the run is over.
    bool iteration_end(RunState& rs) {
        ++rs.iters;
        if (!std::isfinite(history.back())) throw Error(NLTE_E_DIVERGED, "non-finite MALI correction");
        if (stop(history, rs.rho, rs.E)) { rs.status = NLTE_OK; return true; }
        return rs.iters >= max_iterations();
    }

    // After a cycle whose C is in history: the divergence guard (with the fallback to MALI,
    // run here to its end) and the stop rule.  True when the run is over.
    bool cycle_end(RunState& rs) {
        rs.first = false;
        ++rs.cycles;
        const char* why = diverging(rs.grow_run);
        if (why) {
            if (!params.fallback_mali) throw Error(NLTE_E_DIVERGED, why);
            if (log_enabled()) log_line("cycle %d: %s; continuing with MALI", rs.cycles, why);
            fallback_to_mali(rs);
            return true;
        }
        const bool done = stop(history, rs.rho, rs.E);
        if (log_enabled()) log_line("cycle %d: C = %.3e  rho = %.3e  E = %.3e", rs.cycles, history.back(), rs.rho, rs.E);
        if (done) { rs.status = NLTE_OK; return true; }
        return rs.cycles >= max_iterations();
    }

    // Populations from the start of the failing cycle, then plain MALI on the finest grid
    // under the same stop rule, over its own corrections.
    void fallback_to_mali(RunState& rs) {
        Level& F = *lev[nlev - 1];
        dcopy(nprev.as<double>(), F.n.as<double>(), size_t(N) * F.nvox);
        F.fs_valid = false;
        rs.fell_back = 1;
        rs.status = NLTE_W_NOT_CONVERGED;
        rs.rho = rs.E = INFINITY;
        std::vector<double> hm;
        for (int it = 0; it < max_iterations(); ++it) {
            mali(nlev - 1, 1);
            hm.push_back(read_scalar());
            history.push_back(hm.back());
            ++rs.iters;
            if (!std::isfinite(hm.back())) throw Error(NLTE_E_DIVERGED, "non-finite MALI correction after the fallback");
            if (stop(hm, rs.rho, rs.E)) { rs.status = NLTE_OK; break; }
        }
    }

    void run(nlte_result* out) override {
        RunState rs;
        const int top = nlev - 1;
        Level& F = *lev[top];
        const int maxit = max_iterations();
        if (is_mali()) {
            for (int it = 0; it < maxit; ++it) {
                if (params.graph && it > 0) replay([&]() { mali(top, 1); });
                else mali(top, 1);
                history.push_back(read_scalar());
                if (iteration_end(rs)) break;
            }
        } else {
            if (params.method == NLTE_FMG) {
                fmg_prologue();
                rs.first = false;
            }
            for (int c = 0; c < maxit; ++c) {
                if (params.graph && !rs.first) {
                    replay([&]() {
                        dcopy(F.n.as<double>(), nprev.as<double>(), size_t(N) * F.nvox);
                        vcycle(top, false);
                        cycle_change_enqueue(top);
                    });
                    history.push_back(read_scalar());
                } else {
                    dcopy(F.n.as<double>(), nprev.as<double>(), size_t(N) * F.nvox);
                    vcycle(top, rs.first);
                    history.push_back(cycle_change(top));
                }
                if (cycle_end(rs)) break;
            }
        }
        finish(rs, out);
    }

    // The result of a run: final checks and counters.
    void finish(const RunState& rs, nlte_result* out) {
        check_finite(nlev - 1);
        ev_resolve();
        unsigned long long rep = 0;
        HIPCHK(hipMemcpyAsync(&rep, repairs.p, sizeof(rep), hipMemcpyDeviceToHost, st()));
        HIPCHK(hipStreamSynchronize(st()));
        auto t1 = std::chrono::steady_clock::now();
        nlte_result r{};
        r.status = rs.status;
        r.iterations = rs.iters;
        r.cycles = rs.cycles;
        r.C = history.empty() ? 0.0 : history.back();
        r.rho = rs.rho;
        r.E_est = rs.E;
        r.repairs = (long long)rep;
        for (int k = 0; k < nlev && k < 8; ++k) r.formal_solutions[k] = lev[k]->fs_count;
        r.fine_fs_equiv = cost_units;
        r.updates = updates;
        r.ms_total = std::chrono::duration<double, std::milli>(t1 - rs.t0).count();
        r.ms_setup = ms_setup;
        r.ms_sweep = ms_phase[EV_SWEEP];
        r.ms_rates = ms_phase[EV_RATES];
        r.ms_transfer = ms_phase[EV_TRANSFER];
        r.sweep_launches = sweep_launches;
        r.dirs_per_block = fine_db;
        r.sweep_kernel = NLTE_SWEEP_PLANE_STEP;
        r.fallback = rs.fell_back;
        res = r;
        if (out) *out = r;
    }

    // --------------------------------------------------------------- hooks
    Level& level_ref(int level) {
        REQUIRE(level >= 0 && level < nlev, "level out of range");
        return *lev[level];
    }

    static hipMemcpyKind kind_to(int mem) { return mem == NLTE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }
    static hipMemcpyKind kind_from(int mem) { return mem == NLTE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }

    void formal_solution_out(int level, void* jeff, void* oml, int mem) override {
        Level& L = level_ref(level);
        formal_solution(level);
        // direction-group slots summed on the host side of the copy, by the same tree
        // as the rate equations
        const size_t m = size_t(nline) * L.nvox;
        const size_t ns = size_t(L.nslot);
        std::vector<R> a(size_t(2) * ns * m);
        HIPCHK(hipMemcpyAsync(a.data(), L.acc.p, sizeof(R) * a.size(), hipMemcpyDeviceToHost, st()));
        HIPCHK(hipStreamSynchronize(st()));
        std::vector<R> j(m), o(m);
        for (size_t i = 0; i < m; ++i) {
            j[i] = tree_slots(a.data() + i, m, L.nslot);
            o[i] = tree_slots(a.data() + size_t(L.nslot) * m + i, m, L.nslot);
        }
        if (mem == NLTE_MEM_DEVICE) {
            HIPCHK(hipMemcpyAsync(jeff, j.data(), sizeof(R) * m, hipMemcpyHostToDevice, st()));
            HIPCHK(hipMemcpyAsync(oml, o.data(), sizeof(R) * m, hipMemcpyHostToDevice, st()));
            HIPCHK(hipStreamSynchronize(st()));
        } else {
            std::memcpy(jeff, j.data(), sizeof(R) * m);
            std::memcpy(oml, o.data(), sizeof(R) * m);
        }
    }

    // One rate solve from given J-bar^eff and 1 - Lambda* (slot 0 of a two-slot layout, slot 1
    // zero, so the slot sum is the given value exactly).
    double rate_solve_hook(int level, const void* jeff, const void* oml, int mem) override {
        Level& L = level_ref(level);
        REQUIRE(!info.cont_active, "the rate-solve hook takes line radiation only (no active continua)");
        const size_t m = size_t(nline) * L.nvox;
        REQUIRE(L.acc.bytes >= sizeof(R) * 4 * m, "accumulator too small for the rate-solve hook");
        R* acc = L.acc.as<R>();
        HIPCHK(hipMemcpyAsync(acc, jeff, sizeof(R) * m, kind_from(mem), st()));
        HIPCHK(hipMemsetAsync(acc + m, 0, sizeof(R) * m, st()));
        HIPCHK(hipMemcpyAsync(acc + 2 * m, oml, sizeof(R) * m, kind_from(mem), st()));
        HIPCHK(hipMemsetAsync(acc + 3 * m, 0, sizeof(R) * m, st()));
        rate_launch(level, 0, nullptr, nullptr, 0.0, true, true);
        L.fs_valid = false;
        return read_scalar();
    }

    double mali_hook(int level, int iters) override {
        level_ref(level);
        if (iters <= 0) return 0.0;
        mali(level, iters);
        return read_scalar();
    }

    void residual_out(int level, double* dst, int mem) override {
        Level& L = level_ref(level);
        if (!L.fs_valid) formal_solution(level);
        apply_W(level, L.f.as<double>(), L.tmp.as<double>(), -1.0);
        HIPCHK(hipMemcpyAsync(dst, L.tmp.p, sizeof(double) * N * L.nvox, kind_to(mem), st()));
        HIPCHK(hipStreamSynchronize(st()));
    }

    void vcycle_hook(int level, int first) override {
        level_ref(level);
        vcycle(level, first != 0);
        HIPCHK(hipStreamSynchronize(st()));
    }

    // Counters and phase times accumulated so far, also over stage hooks.
    void stats(nlte_result* out) override {
        ev_resolve();
        nlte_result r = res;
        r.C = history.empty() ? 0.0 : history.back();
        r.repairs = repair_count();
        for (int k = 0; k < nlev && k < 8; ++k) r.formal_solutions[k] = lev[k]->fs_count;
        r.fine_fs_equiv = cost_units;
        r.updates = updates;
        r.ms_setup = ms_setup;
        r.ms_sweep = ms_phase[EV_SWEEP];
        r.ms_rates = ms_phase[EV_RATES];
        r.ms_transfer = ms_phase[EV_TRANSFER];
        r.sweep_launches = sweep_launches;
        r.dirs_per_block = fine_db;
        *out = r;
    }

    long long repair_count() override {
        unsigned long long rep = 0;
        HIPCHK(hipMemcpyAsync(&rep, repairs.p, sizeof(rep), hipMemcpyDeviceToHost, st()));
        HIPCHK(hipStreamSynchronize(st()));
        return (long long)rep;
    }

    void get_pops(int level, double* dst, int mem) override {
        Level& L = level_ref(level);
        HIPCHK(hipMemcpyAsync(dst, L.n.p, sizeof(double) * N * L.nvox, kind_to(mem), st()));
        HIPCHK(hipStreamSynchronize(st()));
    }

    void set_pops(int level, const double* src, int mem) override {
        Level& L = level_ref(level);
        HIPCHK(hipMemcpyAsync(L.n.p, src, sizeof(double) * N * L.nvox, kind_from(mem), st()));
        HIPCHK(hipStreamSynchronize(st()));
        L.fs_valid = false;
    }

    void source_function(double* dst, int mem) override {
        Level& F = *lev[nlev - 1];
        DevBuf tmpS;
        double* target = dst;
        if (mem != NLTE_MEM_DEVICE) {
            dalloc(tmpS, sizeof(double) * nline * F.nvox);
            target = tmpS.as<double>();
        }
        source_function_kernel<<<blocks_for(F.nvox, 256), 256, 0, st()>>>(atom_d.as<AtomInfo>(), F.n.as<double>(),
                                                                          target, F.nvox);
        HIPCHK(hipGetLastError());
        if (mem != NLTE_MEM_DEVICE)
            HIPCHK(hipMemcpyAsync(dst, target, sizeof(double) * nline * F.nvox, hipMemcpyDeviceToHost, st()));
        HIPCHK(hipStreamSynchronize(st()));
    }

    void emergent(int ndir, const double* mu, float* dst, int mem) override {
        Level& F = *lev[nlev - 1];
        check_mu(ndir, mu);
        if (!estate.p) dalloc(estate, sizeof(double) * 2 * 3 * size_t(nf) * F.nxy);
        DevBuf o;
        float* target = dst;
        if (mem != NLTE_MEM_DEVICE) {
            dalloc(o, sizeof(float) * size_t(ndir) * nf * F.nxy);
            target = o.as<float>();
        }
        emergent_launch(ndir, mu, target, estate.as<double>(), nf);
        if (mem != NLTE_MEM_DEVICE)
            HIPCHK(hipMemcpyAsync(dst, target, sizeof(float) * size_t(ndir) * nf * F.nxy, hipMemcpyDeviceToHost, st()));
        HIPCHK(hipStreamSynchronize(st()));
    }

    // The same computation with the plane state in a caller-provided device area of
    // `state_bytes` (no allocation): frequencies in chunks whose state fits it.
    void emergent_into(int ndir, const double* mu, float* dst, double* state, size_t state_bytes) override {
        Level& F = *lev[nlev - 1];
        check_mu(ndir, mu);
        const size_t per_f = sizeof(double) * 2 * 3 * F.nxy;
        const int fn = int(std::min<size_t>(size_t(nf), state_bytes / per_f));
        REQUIRE(fn >= 1, "plane of " + std::to_string(F.nxy) + " points too large for the " +
                             std::to_string(state_bytes >> 20) + " MiB emergent-intensity scratch");
        emergent_launch(ndir, mu, dst, state, fn);
        HIPCHK(hipStreamSynchronize(st()));
    }

    void check_mu(int ndir, const double* mu) const {
        for (int d = 0; d < ndir; ++d) {
            const double m[3] = {mu[3 * d], mu[3 * d + 1], mu[3 * d + 2]};
            const double nrm = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
            REQUIRE(nrm > 0 && m[2] / nrm > 1e-6, "emergent directions must point upward");
        }
    }

    // Upward formal solution for each direction at the finest populations, frequencies in
    // chunks of fn (their plane state [2][3][fn][nxy] in `state`); I of the top plane to
    // out[d][f][nxy].  Every frequency is independent, so the chunking does not change it.
    void emergent_launch(int ndir, const double* mu, float* out, double* state, int fn) {
        Level& F = *lev[nlev - 1];
        line_coef_kernel<R><<<blocks_for(F.nvox, 256), 256, 0, st()>>>(atom_d.as<AtomInfo>(), F.n.as<double>(),
                                                                      F.lc.as<R>(), F.nvox);
        HIPCHK(hipGetLastError());
        for (int d = 0; d < ndir; ++d) {
            const double m[3] = {mu[3 * d], mu[3 * d + 1], mu[3 * d + 2]};
            const double nrm = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
            EmergentArgs<R> a;
            a.atom = atom_d.as<AtomInfo>();
            a.nx = F.nx; a.ny = F.ny; a.nz = F.nz; a.nf = nf;
            a.nxy = F.nxy; a.nvox = F.nvox;
            a.dx = F.dx; a.dy = F.dy;
            a.mux = m[0] / nrm; a.muy = m[1] / nrm; a.muz = m[2] / nrm;
            a.z = F.dz.as<double>();
            a.sc = F.sc.as<R>(); a.sv = F.sv.as<R>(); a.lc = F.lc.as<R>(); a.qf = qf.as<R>();
            a.line_of = line_of_d.as<int>();
            a.state = state;
            a.out = out + size_t(d) * nf * F.nxy;
            a.herm = params.sc_interp == NLTE_SC_HERMITE ? 1 : 0;
            for (int f0 = 0; f0 < nf; f0 += fn) {
                a.f0 = f0;
                a.fn = std::min(fn, nf - f0);
                for (int k = 0; k < F.nz; ++k)
                    emergent_step_kernel<R><<<blocks_for(size_t(a.fn) * F.nxy, 256), 256, 0, st()>>>(a, k);
            }
            HIPCHK(hipGetLastError());
        }
    }

    // Emergent intensity at the continuum frequencies (active continua): an upward formal
    // solution per direction in FP64 from the finest populations, I of the top plane to
    // dst[d][nfc][nxy].
    void emergent_continuum(int ndir, const double* mu, float* dst, int mem) override {
        REQUIRE(info.cont_active, "the atom has no active continua");
        Level& F = *lev[nlev - 1];
        check_mu(ndir, mu);
        if (!cestate.p) dalloc(cestate, sizeof(double) * 2 * 3 * size_t(nfc) * F.nxy);
        DevBuf o;
        float* target = dst;
        if (mem != NLTE_MEM_DEVICE) {
            dalloc(o, sizeof(float) * size_t(ndir) * nfc * F.nxy);
            target = o.as<float>();
        }
        for (int d = 0; d < ndir; ++d) {
            const double m[3] = {mu[3 * d], mu[3 * d + 1], mu[3 * d + 2]};
            const double nrm = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
            EmergentContArgs a;
            a.atom = atom_d.as<AtomInfo>();
            a.nx = F.nx; a.ny = F.ny; a.nz = F.nz; a.nfc = nfc;
            a.nxy = F.nxy; a.nvox = F.nvox;
            a.dx = F.dx; a.dy = F.dy;
            a.mux = m[0] / nrm; a.muy = m[1] / nrm; a.muz = m[2] / nrm;
            a.z = F.dz.as<double>();
            a.prim = F.prim.as<double>();
            a.nstar = F.nstar.as<double>();
            a.n = F.n.as<double>();
            a.cnu = cnu_d.as<double>(); a.ce = ce_d.as<double>(); a.calpha = calpha_d.as<double>();
            a.state = cestate.as<double>();
            a.out = target + size_t(d) * nfc * F.nxy;
            for (int k = 0; k < F.nz; ++k)
                emergent_cont_step_kernel<<<blocks_for(size_t(nfc) * F.nxy, 256), 256, 0, st()>>>(a, k);
            HIPCHK(hipGetLastError());
        }
        if (mem != NLTE_MEM_DEVICE)
            HIPCHK(hipMemcpyAsync(dst, target, sizeof(float) * size_t(ndir) * nfc * F.nxy, hipMemcpyDeviceToHost, st()));
        HIPCHK(hipStreamSynchronize(st()));
    }

    void restrict_hook(int level, int nq, const double* src, double* dst) override {
        REQUIRE(level >= 1 && level < nlev, "restriction needs 1 <= level < nlev");
        restrict_fields(level, nq, src, dst);
        HIPCHK(hipStreamSynchronize(st()));
    }

    void prolong_hook(int level, int nq, const double* src, double* dst) override {
        REQUIRE(level >= 1 && level < nlev, "prolongation needs 1 <= level < nlev");
        prolong_fields(level, nq, src, dst);
        HIPCHK(hipStreamSynchronize(st()));
    }
};



// ===================================================================== batches
// Several jobs solved together (small grids underfill the device: Sect. 4.9 notes that
// coarse grids cost more than their share).  Their formal solutions share work-list
// launches - per plane step, one launch per class of frequency chunks over the tiles of
// every job still sweeping (sweep_list_kernel) - and everything else runs per job, all
// on one stream.  The jobs go through the same method schedule in lockstep and each
// leaves the batch when its own stop rule (or cap, or guard) ends its run.  Every job
// computes exactly what it computes alone: each keeps its frequency chunks, and the
// direction sums do not depend on the block shape.
template <typename R>
struct Batch {
    nlte_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    std::vector<Job<R>*> jobs;
    std::vector<typename Job<R>::RunState> rs;
    std::vector<int> done;              // 1 once a job's run has ended
    std::vector<std::string> error;     // message of a job that failed
    std::vector<nlte_status> code;
    // device work lists, cached per (level, job set): per frequency-chunk class the
    // SweepArgs of its jobs, then their first blocks
    struct Table {
        DevBuf buf;
        struct Cls { int fc = 0, n = 0; size_t args = 0, first = 0; std::vector<int> idx, nz; std::vector<unsigned> first_h; };
        std::vector<Cls> cls;
        int maxnz = 0;
    };
    std::map<std::pair<int, std::vector<int>>, std::unique_ptr<Table>> tables;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
    double ms_sweep = 0;
    long long launches = 0;

    // HIP-graph replay of repeated steps, when every job asked for it (params.graph): a step
    // (one MALI iteration, or one cycle after the first) of a given job set runs eagerly once,
    // creating its work lists; the next time it is captured, and from then on replayed.  The
    // host bookkeeping of the captured step (formal-solution counts, updates, launches) is
    // recorded at capture and added per replay; replayed work is not timed.
    bool graphs = false;
    bool capturing = false;
    struct Book {
        std::vector<long long> fs;   // per level
        double cost = 0, upd = 0;
        long long launches = 0;
    };
    struct Replay {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        std::vector<Book> delta;      // per job of the set
        long long launches = 0;       // the batch's own launch count
        bool eager_only = false;      // capture failed once: this step stays eager
    };
    std::map<std::pair<std::vector<int>, int>, Replay> replays;
    std::map<std::pair<std::vector<int>, int>, int> eager_runs;

    ~Batch() {
        for (auto& e : evs) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
        for (auto& r : replays) drop(r.second);
    }

    static void drop(Replay& r) {
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
        r.exec = nullptr;
        r.graph = nullptr;
    }

    Book book(int j) const {
        const Job<R>& J = *jobs[j];
        Book b;
        for (auto& L : J.lev) b.fs.push_back(L->fs_count);
        b.cost = J.cost_units;
        b.upd = J.updates;
        b.launches = J.sweep_launches;
        return b;
    }

    void set_book(int j, const Book& b) {
        Job<R>& J = *jobs[j];
        for (size_t k = 0; k < J.lev.size(); ++k) J.lev[k]->fs_count = b.fs[k];
        J.cost_units = b.cost;
        J.updates = b.upd;
        J.sweep_launches = b.launches;
    }

    // Runs `work` for the jobs in `set`: eagerly, or as a captured graph (see `graphs`).
    template <typename F>
    void run_step(const std::vector<int>& set, int kind, bool repeatable, F&& work) {
        if (!graphs || !repeatable) {
            work();
            return;
        }
        const auto key = std::make_pair(set, kind);
        Replay& r = replays[key];
        if (r.eager_only || eager_runs[key] < 1) {
            work();
            ++eager_runs[key];
            return;
        }
        if (!r.exec) {
            std::vector<Book> before;
            for (int j : set) before.push_back(book(j));
            const long long l0 = launches;
            for (int j : set) jobs[j]->capturing = true;
            capturing = true;
            bool ok = true;
            HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            try {
                work();
            } catch (...) {
                ok = false;
            }
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(stream, &g);
            capturing = false;
            for (int j : set) jobs[j]->capturing = false;
            if (ok && ec == hipSuccess && g && hipGraphInstantiate(&r.exec, g, nullptr, nullptr, 0) == hipSuccess) {
                r.graph = g;
                r.delta.clear();
                for (size_t i = 0; i < set.size(); ++i) {
                    const Book after = book(set[i]);
                    Book d;
                    for (size_t k = 0; k < after.fs.size(); ++k) d.fs.push_back(after.fs[k] - before[i].fs[k]);
                    d.cost = after.cost - before[i].cost;
                    d.upd = after.upd - before[i].upd;
                    d.launches = after.launches - before[i].launches;
                    r.delta.push_back(d);
                    set_book(set[i], before[i]);
                }
                r.launches = launches - l0;
                launches = l0;
            } else {
                // nothing ran on the device: undo the host bookkeeping and run eagerly
                (void)hipGetLastError();
                if (g) (void)hipGraphDestroy(g);
                r.exec = nullptr;
                r.eager_only = true;
                for (size_t i = 0; i < set.size(); ++i) set_book(set[i], before[i]);
                launches = l0;
                work();
                return;
            }
        }
        HIPCHK(hipGraphLaunch(r.exec, stream));
        for (size_t i = 0; i < set.size(); ++i) {
            Book b = book(set[i]);
            for (size_t k = 0; k < b.fs.size(); ++k) b.fs[k] += r.delta[i].fs[k];
            b.cost += r.delta[i].cost;
            b.upd += r.delta[i].upd;
            b.launches += r.delta[i].launches;
            set_book(set[i], b);
        }
        launches += r.launches;
    }

    static int class_db(int fc) { return list_block_dirs(sizeof(R), fc); }

    Table& table(int k, const std::vector<int>& set) {
        auto key = std::make_pair(k, set);
        auto it = tables.find(key);
        if (it != tables.end()) return *it->second;
        if (capturing) throw Error(NLTE_E_INVALID, "work list missing during graph capture");
        auto t = std::make_unique<Table>();
        std::vector<SweepArgs<R>> args;
        for (int fc : {1, 2, 4}) {
            typename Table::Cls c;
            c.fc = fc;
            std::vector<std::pair<int, int>> order;   // (nz, job) for the jobs of this class
            for (int j : set)
                if (jobs[j]->lev[k]->fc == fc) order.push_back({jobs[j]->lev[k]->nz, j});
            if (order.empty()) continue;
            std::stable_sort(order.begin(), order.end(), [](auto& a, auto& b) { return a.first > b.first; });
            const int db = class_db(fc);
            c.first_h.push_back(0);
            for (auto& o : order) {
                const Level& L = *jobs[o.second]->lev[k];
                c.idx.push_back(o.second);
                c.nz.push_back(L.nz);
                c.first_h.push_back(c.first_h.back() + unsigned((L.nxy + 63) / 64) * unsigned(jobs[o.second]->nline) *
                                                           unsigned(kNDir / db));
                t->maxnz = std::max(t->maxnz, L.nz);
            }
            c.n = int(order.size());
            t->cls.push_back(c);
        }
        // one device buffer: every class's SweepArgs array, then its first-block array
        size_t bytes = 0;
        for (auto& c : t->cls) {
            c.args = bytes;
            bytes += sizeof(SweepArgs<R>) * c.n;
            bytes = (bytes + 255) & ~size_t(255);
            c.first = bytes;
            bytes += sizeof(unsigned) * (c.n + 1);
            bytes = (bytes + 255) & ~size_t(255);
        }
        std::vector<unsigned char> host(bytes, 0);
        for (auto& c : t->cls) {
            for (int i = 0; i < c.n; ++i) {
                SweepArgs<R> a = jobs[c.idx[i]]->sweep_args(k);
                a.m0 = 0;
                a.Q = jobs[c.idx[i]]->Qpass;
                a.add = 0;
                std::memcpy(host.data() + c.args + sizeof(SweepArgs<R>) * i, &a, sizeof(a));
            }
            std::memcpy(host.data() + c.first, c.first_h.data(), sizeof(unsigned) * (c.n + 1));
        }
        t->buf.alloc(ctx, bytes);
        HIPCHK(hipMemcpyAsync(t->buf.p, host.data(), bytes, hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));   // host is a temporary
        Table& ref = *t;
        tables[key] = std::move(t);
        return ref;
    }

    template <int DB>
    void launch(const Table& t, const typename Table::Cls& c, int nact, int s) {
        const auto* a = reinterpret_cast<const SweepArgs<R>*>(static_cast<const unsigned char*>(t.buf.p) + c.args);
        const auto* f = reinterpret_cast<const unsigned*>(static_cast<const unsigned char*>(t.buf.p) + c.first);
        sweep_list_kernel<R, DB><<<c.first_h[nact], unsigned(DB * c.fc * 64), 0, stream>>>(a, f, nact, s);
    }

    // One formal solution of level k for the jobs in `set`.
    void formal_solution(int k, const std::vector<int>& set) {
        if (set.empty()) return;
        Table& t = table(k, set);
        for (int j : set) jobs[j]->line_coef(k);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (!capturing) {
            HIPCHK(hipEventCreate(&e0));
            HIPCHK(hipEventCreate(&e1));
            evs.push_back({e0, e1});
            HIPCHK(hipEventRecord(e0, stream));
        }
        for (int s = 0; s < t.maxnz; ++s)
            for (auto& c : t.cls) {
                int nact = 0;
                while (nact < c.n && c.nz[nact] > s) ++nact;
                if (!nact) continue;
                switch (class_db(c.fc)) {
                    case 12: launch<12>(t, c, nact, s); break;
                    case 6: launch<6>(t, c, nact, s); break;
                    default: launch<3>(t, c, nact, s); break;
                }
                ++launches;
            }
        HIPCHK(hipGetLastError());
        if (!capturing) HIPCHK(hipEventRecord(e1, stream));
        for (auto& c : t.cls)
            for (int i = 0; i < c.n; ++i) jobs[c.idx[i]]->list_finish(k, class_db(c.fc), c.nz[i]);
    }

    // iters[j] MALI iterations on level k for the jobs in `set`.
    void mali(int k, const std::vector<int>& set, const std::vector<int>& iters) {
        int most = 0;
        for (int j : set) most = std::max(most, iters[j]);
        for (int it = 0; it < most; ++it) {
            std::vector<int> part, need;
            for (int j : set)
                if (iters[j] > it) {
                    part.push_back(j);
                    if (!(it == 0 && jobs[j]->lev[k]->fs_valid)) need.push_back(j);
                }
            formal_solution(k, need);
            for (int j : part) {
                jobs[j]->rate_launch(k, 0, nullptr, nullptr, 0.0, true);
                jobs[j]->lev[k]->fs_valid = false;
            }
        }
    }

    std::vector<int> all(int n) const { return std::vector<int>(jobs.size(), n); }

    // One FAS V-cycle on levels k..0 for the jobs in `set` (the same steps as Job::vcycle).
    void vcycle(int k, const std::vector<int>& set, const std::vector<char>& first) {
        const nlte_params& p = jobs[set[0]]->params;
        std::vector<int> pre(jobs.size(), 0);
        for (int j : set) pre[j] = (first[j] && p.nu0 > 0) ? p.nu0 : p.nu1;
        if (k == 0) {
            mali(0, set, pre);
            mali(0, set, all(p.nu2));
            return;
        }
        mali(k, set, pre);
        std::vector<int> need;
        for (int j : set)
            if (!jobs[j]->lev[k]->fs_valid) need.push_back(j);
        formal_solution(k, need);
        for (int j : set) jobs[j]->vc_restrict(k);
        formal_solution(k - 1, set);
        for (int j : set) jobs[j]->vc_coarse_rhs(k);
        if (k - 1 == 0) mali(0, set, all(p.nu3));
        else vcycle(k - 1, set, std::vector<char>(jobs.size(), 0));
        for (int j : set) jobs[j]->vc_correct(k);
        mali(k, set, all(p.nu2));
    }

    // Ends job j's run: result into out[j], or the error that stopped it.
    template <typename F>
    void guarded_step(int j, F&& fn) {
        try {
            fn();
        } catch (const Error& e) {
            done[j] = 1;
            code[j] = e.code;
            error[j] = e.what();
        } catch (const std::exception& e) {
            done[j] = 1;
            code[j] = NLTE_E_INVALID;
            error[j] = e.what();
        }
    }

    // Adds jobs (built, with their initial populations) to the batch; returns their indices.
    std::vector<int> add(const std::vector<Job<R>*>& js) {
        std::vector<int> idx;
        for (Job<R>* j : js) {
            idx.push_back(int(jobs.size()));
            jobs.push_back(j);
            rs.emplace_back();
            done.push_back(0);
            error.emplace_back();
            code.push_back(NLTE_OK);
            out.emplace_back();
        }
        return idx;
    }

    std::vector<int> active() const {
        std::vector<int> a;
        for (size_t j = 0; j < jobs.size(); ++j)
            if (!done[j]) a.push_back(int(j));
        return a;
    }

    std::vector<nlte_result> out;   // per job, valid once done

    // The start of newly added jobs' runs: full multigrid from their coarsest grids (FMG;
    // Sect. 2.3), else nothing (FAS starts with a first cycle, MALI with an iteration).
    void start(const std::vector<int>& set) {
        if (set.empty()) return;
        Job<R>& j0 = *jobs[set[0]];
        if (j0.is_mali() || j0.params.method != NLTE_FMG) return;
        const int top = j0.nlev - 1;
        mali(0, set, all(j0.params.nu_fmg));
        for (int k = 1; k <= top; ++k) {
            for (int j : set) {
                jobs[j]->prolong_fields(k, jobs[j]->N, jobs[j]->lev[k - 1]->n.template as<double>(),
                                        jobs[j]->lev[k]->n.template as<double>());
                jobs[j]->lev[k]->fs_valid = false;
            }
            if (k < top) vcycle(k, set, std::vector<char>(jobs.size(), 0));
        }
        for (int j : set) rs[j].first = false;
    }

    // One cycle (FAS/FMG) or MALI iteration of the jobs in `set`; returns the jobs whose
    // runs ended with it (their results in out[], or their errors).
    std::vector<int> step(const std::vector<int>& set) {
        std::vector<int> ended;
        if (set.empty()) return ended;
        Job<R>& j0 = *jobs[set[0]];
        const int top = j0.nlev - 1;
        const bool m = j0.is_mali();
        if (m) {
            run_step(set, 0, true, [&]() { mali(top, set, all(1)); });
        } else {
            std::vector<char> first(jobs.size(), 0);
            bool any_first = false;
            for (int j : set) {
                first[j] = rs[j].first ? 1 : 0;
                any_first = any_first || first[j];
            }
            run_step(set, 1, !any_first, [&]() {
                for (int j : set) {
                    Level& F = *jobs[j]->lev[top];
                    jobs[j]->dcopy(F.n.template as<double>(), jobs[j]->nprev.template as<double>(),
                                   size_t(jobs[j]->N) * F.nvox);
                }
                vcycle(top, set, first);
                for (int j : set) jobs[j]->cycle_change_enqueue(top);
            });
        }
        for (int j : set) {
            bool over = false;
            guarded_step(j, [&]() {
                jobs[j]->history.push_back(jobs[j]->read_scalar());
                over = m ? jobs[j]->iteration_end(rs[j]) : jobs[j]->cycle_end(rs[j]);
            });
            if (done[j]) {            // failed
                ended.push_back(j);
                continue;
            }
            if (over) {
                guarded_step(j, [&]() { jobs[j]->finish(rs[j], &out[j]); });
                done[j] = 1;
                ended.push_back(j);
            }
        }
        // graphs of job sets with an ended job never run again
        if (!ended.empty())
            for (auto it = replays.begin(); it != replays.end();) {
                bool stale = false;
                for (int j : it->first.first)
                    stale = stale || std::find(ended.begin(), ended.end(), j) != ended.end();
                if (stale) {
                    drop(it->second);
                    eager_runs.erase(it->first);
                    it = replays.erase(it);
                } else {
                    ++it;
                }
            }
        // sweep time of the batch so far (events resolved as they complete)
        HIPCHK(hipStreamSynchronize(stream));
        for (auto& e : evs) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
            ms_sweep += ms;
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        evs.clear();
        for (int j : ended) {
            if (code[j] < 0) {
                out[j] = nlte_result{};
                out[j].status = code[j];
            }
            out[j].ms_sweep = ms_sweep;   // the batch's sweep time so far, shared by its jobs
            if (code[j] >= 0) jobs[j]->res = out[j];
        }
        return ended;
    }

    void run(nlte_result* res) {
        start(active());
        for (std::vector<int> a = active(); !a.empty(); a = active()) step(a);
        for (size_t j = 0; j < jobs.size(); ++j) res[j] = out[j];
    }
};

// True when job j can run in a batch with job a (built jobs).
template <typename R>
bool batchable(const Job<R>& a, const Job<R>& j) {
    const nlte_params& p = j.params;
    const nlte_params& q = a.params;
    if (p.method != q.method || j.nlev != a.nlev || p.nu_fmg != q.nu_fmg || p.nu0 != q.nu0 || p.nu1 != q.nu1 ||
        p.nu2 != q.nu2 || p.nu3 != q.nu3 || (p.graph != 0) != (q.graph != 0))
        return false;
    for (int k = 0; k < j.nlev; ++k)
        if (!j.list_sweep_ok(k)) return false;
    return true;
}

// Checks that jobs can share a batch, and runs it.
template <typename R>
nlte_status run_batch(nlte_ctx* ctx, const std::vector<JobBase*>& in, hipStream_t stream, nlte_result* out,
                      std::string* first_error) {
    std::vector<Job<R>*> js;
    for (JobBase* jb : in) {
        auto* j = dynamic_cast<Job<R>*>(jb);
        REQUIRE(j, "a batch takes jobs of one precision");
        js.push_back(j);
    }
    for (Job<R>* j : js) REQUIRE(batchable(*js[0], *j), "a batch takes jobs of one method, number of grids and "
                                                         "iteration counts, with plane-step bilinear sweeps in "
                                                         "one frequency pass, no active continua, and graph "
                                                         "replay asked for by all of them or by none");
    // Graph capture needs a stream of its own (the context's may be the null stream): the
    // batch then runs on a private stream that follows the context's and that the
    // context's stream waits for at the end.
    struct Private {
        hipStream_t parent = nullptr, s = nullptr;
        hipEvent_t ev = nullptr;
        ~Private() {
            if (!s) {
                if (ev) (void)hipEventDestroy(ev);
                return;
            }
            if (hipEventRecord(ev, s) == hipSuccess) (void)hipStreamWaitEvent(parent, ev, 0);
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
            (void)hipEventDestroy(ev);
        }
    } priv;
    const bool graphs = !in.empty() && in[0]->params.graph != 0;
    hipStream_t bs = stream;
    if (graphs) {
        priv.parent = stream;
        HIPCHK(hipEventCreateWithFlags(&priv.ev, hipEventDisableTiming));
        HIPCHK(hipStreamCreateWithFlags(&priv.s, hipStreamNonBlocking));
        HIPCHK(hipEventRecord(priv.ev, stream));
        HIPCHK(hipStreamWaitEvent(priv.s, priv.ev, 0));
        bs = priv.s;
    }
    Batch<R> b;
    b.ctx = ctx;
    b.stream = bs;
    b.graphs = graphs;
    b.add(js);
    for (Job<R>* j : b.jobs) j->batch_stream = bs;
    try {
        b.run(out);
    } catch (...) {
        for (Job<R>* j : b.jobs) j->batch_stream = nullptr;
        throw;
    }
    for (Job<R>* j : b.jobs) j->batch_stream = nullptr;
    nlte_status worst = NLTE_OK;
    for (size_t j = 0; j < b.jobs.size(); ++j)
        if (b.code[j] < 0) {
            if (worst >= 0) {
                worst = b.code[j];
                if (first_error) *first_error = "job " + std::to_string(j) + ": " + b.error[j];
            }
        }
    return worst;
}

// Device bytes a job will allocate (same formulas as Job::build; the emergent-intensity
// state is included so that an admitted job never exceeds its reservation).
size_t job_footprint(const nlte_ctx* ctx, const nlte_atmos* atm, const nlte_atom* atom, const nlte_params* p) {
    const size_t R = p->precision == NLTE_FP64 ? 8 : 4;
    const int nline = atom->info.nline, N = atom->info.N, nf = atom->nf;
    const int nlev = std::max(1, p->method == NLTE_MALI ? 1 : p->nlev);
    const int nprim = 7 + atm->nline_chic;
    const size_t cell = R == 8 ? sizeof(Cell<double>) : sizeof(Cell<float>);
    size_t bytes = sizeof(AtomInfo) + (2 * R + 4) * size_t(nf) + 64;
    int nx = atm->nx, ny = atm->ny, nz = atm->nz;
    size_t fine_nxy = size_t(nx) * ny, fine_nvox = fine_nxy * nz;
    int maxfreq = 0;
    for (int l = 0; l < nline; ++l) maxfreq = std::max(maxfreq, atom->info.line[l].nfreq);
    for (int k = nlev - 1; k >= 0; --k) {
        const size_t nvox = size_t(nx) * ny * nz;
        const size_t slots = size_t(acc_slots(nvox, nline, R));
        bytes += 8 * size_t(nz) + 8 * size_t(nprim) * nvox + R * (6 * nline + 4) * nvox;
        bytes += 8 * (size_t(N) * 6 + size_t(N) * N + 1) * nvox + R * (2 * slots + 2) * nline * nvox;
        bytes += 8 * std::max<size_t>((nvox + 255) / 256, 1024);
        if (atom->info.cont_active)   // LTE ratios, h/kT, spontaneous rates, U/G/L sums
            bytes += (R * (atom->info.ncont + 1) + 8 * atom->info.ncont +
                      R * (2 + atom->info.cont_nup) * atom->info.ncont * kMaxSlots) * nvox;
        nx /= 2; ny /= 2; nz = (nz - 1) / 2 + 1;
    }
    const char* envb = std::getenv("NLTE3D_SWEEP_STATE_MB");
    const double cap = envb ? std::atof(envb) * 1048576.0 : 0.25 * double(ctx->budget);
    const int nstate = 2;
    const double per_q = double(cell) * nstate * kNDir * nline * fine_nxy;
    int Q = std::max(1, std::min(maxfreq, int(cap / per_q)));
    Q = std::max(1, std::min(Q, int(4294967295.0 / (double(cell) * double(fine_nxy)))));
    bytes += cell * nstate * kNDir * size_t(nline) * Q * fine_nxy;
    bytes += 8 * size_t(N) * fine_nvox;
    // active continua: plane state, frequency tables, and the continuum emergent intensity's
    // state with one direction of its output
    if (atom->info.cont_active)
        bytes += 3 * R * 2 * kNDir * atom->cnu.size() * fine_nxy +
                 8 * (2 + 2 * size_t(atom->info.ncont)) * atom->cnu.size() + R * kContRow * atom->cnu.size() +
                 (8 * 6 + 4) * atom->cnu.size() * fine_nxy;
    if (p->top_I) bytes += R * size_t(nf) * fine_nxy;
    bytes += 8 * 6 * size_t(nf) * fine_nxy;             // emergent-intensity state
    bytes += 4 * size_t(nf) * fine_nxy;                  // one direction of host-bound output
    bytes += 8 * size_t(nline) * fine_nvox;              // source-function staging
    return bytes;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Serving worker: admits the queue head when its footprint fits the unreserved budget
// (submission already checked that it fits an empty context),
// then builds and runs it on its own stream; several workers run jobs concurrently, so
// their kernels overlap on the device and a queued job starts as soon as memory frees.
// A job leaves the queue and becomes RUNNING in one step under qmu, and its final state
// is published last, under qmu, after its times, status and accounting are written:
// nlte_release, which waits under qmu for a final state, then owns the job alone.
// With batching (nlte_serve_batching), the worker runs the head together with queued jobs
// that can share its batch, and admits more of them between cycles as they arrive.

// Takes job j out of the queue as RUNNING with its footprint reserved (qmu held).
static void admit_locked(nlte_ctx* ctx, JobBase* j) {
    ctx->reserved += j->footprint;
    ctx->running++;
    j->t_admit = now_s();
    j->state = NLTE_JOB_RUNNING;
}

// Publishes a finished job (the worker does not touch it afterwards).
static void publish(nlte_ctx* ctx, JobBase* j, int final_state, bool reservation_held) {
    j->t_done = now_s();
    {
        std::lock_guard<std::mutex> lk(ctx->qmu);
        ctx->running--;
        if (reservation_held) ctx->reserved -= j->footprint;
        j->state = final_state;
    }
    ctx->qcv.notify_all();
}

// Served jobs whose parameters let them share a batch (checked again once built).
static bool batch_key_equal(const JobBase* a, const JobBase* b) {
    const nlte_params& p = a->params;
    const nlte_params& q = b->params;
    auto nl = [](const nlte_params& x) { return x.method == NLTE_MALI ? 1 : std::max(1, x.nlev); };
    return a->prec == b->prec && p.method == q.method && nl(p) == nl(q) && p.nu_fmg == q.nu_fmg &&
           p.nu0 == q.nu0 && p.nu1 == q.nu1 && p.nu2 == q.nu2 && p.nu3 == q.nu3 &&
           (p.graph != 0) == (q.graph != 0);
}
// Serving batches exist to fill the device with grids too small to fill it alone.  One
// plane step of 64x64 points x 24 directions x 505 frequencies (49.6 M updates) already
// runs at the full sweep rate, so served jobs share a batch only while their summed
// finest-grid plane-step work stays within that.  A batch advances its jobs in lockstep,
// one formal solution at a time, so a small grid tied to a large one would wait for every
// plane of the large one: only jobs whose finest-grid formal solutions are within a factor
// of 4 of the batch's first job share it.
constexpr double kBatchFill = 64.0 * 64.0 * 24.0 * 505.0;
constexpr double kBatchSpread = 4.0;
static double plane_work(const JobBase* j) {
    return double(j->src_atmos->nx) * double(j->src_atmos->ny) * 24.0 * double(j->src_atom->nf);
}
static double fs_work(const JobBase* j) { return plane_work(j) * double(j->src_atmos->nz); }
static bool batch_similar(const JobBase* a, const JobBase* b) {
    const double r = fs_work(a) / fs_work(b);
    return r <= kBatchSpread && r >= 1.0 / kBatchSpread;
}

static bool batch_candidate(const JobBase* j) {
    const nlte_params& p = j->params;
    return p.sc_interp == NLTE_SC_BILINEAR &&
           (p.sweep_kernel == NLTE_SWEEP_AUTO || p.sweep_kernel == NLTE_SWEEP_PLANE_STEP) &&
           !j->src_atom->info.cont_active && plane_work(j) < kBatchFill;
}

// Admits queued jobs that can join a batch keyed by `ref` and fit the budget, in queue
// order, up to `room` of them and `fill` plane-step work in all (qmu taken here).
static std::vector<JobBase*> admit_joiners(nlte_ctx* ctx, const JobBase* ref, int room, double fill) {
    std::vector<JobBase*> out;
    if (room <= 0) return out;
    std::lock_guard<std::mutex> lk(ctx->qmu);
    for (auto it = ctx->queue.begin(); it != ctx->queue.end() && int(out.size()) < room;) {
        JobBase* q = *it;
        if (batch_candidate(q) && batch_key_equal(ref, q) && batch_similar(ref, q) && plane_work(q) <= fill &&
            ctx->used + ctx->reserved + q->footprint <= ctx->budget) {
            fill -= plane_work(q);
            it = ctx->queue.erase(it);
            admit_locked(ctx, q);
            out.push_back(q);
        } else {
            ++it;
        }
    }
    return out;
}

static void run_alone(nlte_ctx* ctx, JobBase* j, bool reservation_held);

// A serving batch: the head and every compatible job admitted with it or later.
template <typename R>
void serve_batch(nlte_ctx* ctx, JobBase* head) {
    hipStream_t bs = nullptr;
    if (hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        run_alone(ctx, head, true);
        return;
    }
    int bid;
    {
        std::lock_guard<std::mutex> lk(ctx->qmu);
        bid = ctx->next_batch++;
    }
    Batch<R> b;
    b.ctx = ctx;
    b.stream = bs;
    b.graphs = head->params.graph != 0;
    std::vector<JobBase*> pending = {head};
    for (JobBase* q : admit_joiners(ctx, head, ctx->batch_max - 1, kBatchFill - plane_work(head)))
        pending.push_back(q);
    Job<R>* ref = nullptr;
    for (;;) {
        std::vector<Job<R>*> fresh;
        for (JobBase* p : pending) {
            auto* j = static_cast<Job<R>*>(p);
            bool held = true;
            try {
                j->batch_stream = bs;
                j->build_served();
                {
                    std::lock_guard<std::mutex> lk(ctx->qmu);
                    ctx->reserved -= j->footprint;
                    held = false;
                }
                if (ref && !batchable(*ref, *j)) {   // found unsuited once built: alone, here
                    j->batch_stream = nullptr;
                    run_alone(ctx, j, false);
                    continue;
                }
                if (!ref) {
                    if (!batchable(*j, *j)) {
                        j->batch_stream = nullptr;
                        run_alone(ctx, j, false);
                        continue;
                    }
                    ref = j;
                }
                j->batch_id = bid;
                fresh.push_back(j);
            } catch (const Error& e) {
                j->batch_stream = nullptr;
                j->final_status = e.code;
                j->error = e.what();
                publish(ctx, j, NLTE_JOB_FAILED, held);
            } catch (const std::exception& e) {
                j->batch_stream = nullptr;
                j->final_status = NLTE_E_INVALID;
                j->error = e.what();
                publish(ctx, j, NLTE_JOB_FAILED, held);
            }
        }
        pending.clear();
        std::vector<int> ended;
        try {
            b.start(b.add(fresh));
            ended = b.step(b.active());
        } catch (const std::exception& e) {   // the batch as a whole failed: fail its jobs
            const nlte_status c = dynamic_cast<const Error*>(&e) ? static_cast<const Error&>(e).code : NLTE_E_DEVICE;
            for (int j : b.active()) {
                b.done[j] = 1;
                b.code[j] = c;
                b.error[j] = e.what();
                ended.push_back(j);
            }
        }
        for (int j : ended) {
            Job<R>* job = b.jobs[j];
            job->batch_stream = nullptr;
            if (b.code[j] < 0) {
                job->final_status = b.code[j];
                job->error = b.error[j];
                publish(ctx, job, NLTE_JOB_FAILED, false);
            } else {
                job->final_status = b.out[j].status;
                publish(ctx, job, NLTE_JOB_DONE, false);
            }
        }
        const std::vector<int> act = b.active();
        const int live = int(act.size());
        double fill = kBatchFill;
        for (int i : act) fill -= plane_work(b.jobs[i]);
        if (ref && !ctx->stopping) pending = admit_joiners(ctx, ref, ctx->batch_max - live, fill);
        if (live == 0 && pending.empty()) break;
    }
    (void)hipStreamSynchronize(bs);
    (void)hipStreamDestroy(bs);
}

static void run_alone(nlte_ctx* ctx, JobBase* j, bool reservation_held) {
    int final_state = NLTE_JOB_DONE;
    try {
        if (!j->own_stream) HIPCHK(hipStreamCreateWithFlags(&j->own_stream, hipStreamNonBlocking));
        if (reservation_held) {
            j->build_served();
            {   // the job's buffers now count in `used`; drop the reservation
                std::lock_guard<std::mutex> lk(ctx->qmu);
                ctx->reserved -= j->footprint;
                reservation_held = false;
            }
        }
        nlte_result r{};
        j->run(&r);
        j->final_status = r.status;
    } catch (const Error& e) {
        j->final_status = e.code;
        j->error = e.what();
        final_state = NLTE_JOB_FAILED;
    } catch (const std::exception& e) {
        j->final_status = NLTE_E_INVALID;
        j->error = e.what();
        final_state = NLTE_JOB_FAILED;
    }
    publish(ctx, j, final_state, reservation_held);
}

void serve_worker(nlte_ctx* ctx) {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        JobBase* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(ctx->qmu);
            for (;;) {
                if (ctx->stopping) return;
                if (!ctx->queue.empty()) {
                    JobBase* head = ctx->queue.front();
                    // memory of finished jobs counts until they are released
                    const bool fits = ctx->used + ctx->reserved + head->footprint <= ctx->budget;
                    if (fits) {
                        ctx->queue.pop_front();
                        admit_locked(ctx, head);
                        j = head;
                        break;
                    }
                }
                ctx->qcv.wait(lk);
            }
        }
        if (ctx->batch_max > 1 && batch_candidate(j)) {
            if (j->prec == NLTE_FP64) serve_batch<double>(ctx, j);
            else serve_batch<float>(ctx, j);
        } else {
            run_alone(ctx, j, true);
        }
    }
}

// ------------------------------------------------------------------ API helpers
template <typename F>
nlte_status guarded(nlte_ctx* ctx, F&& fn) {
    if (!ctx) return NLTE_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        nlte_status s = fn();
        if (s >= 0) ctx->err.clear();
        return s;
    } catch (const Error& e) {
        ctx->err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return NLTE_E_OOM;
    } catch (const std::exception& e) {
        ctx->err = e.what();
        return NLTE_E_INVALID;
    }
}

JobBase* find_job(nlte_ctx* ctx, nlte_job job, bool need_done = true) {
    auto it = ctx->jobs.find(job);
    if (it == ctx->jobs.end()) throw Error(NLTE_E_INVALID, "unknown job handle");
    JobBase* j = it->second;
    if (need_done && j->served && j->state < 2) throw Error(NLTE_E_INVALID, "job not finished");
    if (need_done && j->served && j->state == 3) throw Error(NLTE_E_INVALID, "job failed: " + j->error);
    return j;
}

bool finite_host(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

// ===================================================================== C-ABI
extern "C" {

const char* nlte_version(void) { return "nlte3d 0.1 (gfx950)"; }

nlte_status nlte_ctx_create(int device, void* hip_stream, size_t hbm_budget, nlte_ctx** out) {
    if (!out) return NLTE_E_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return NLTE_E_DEVICE;
    if (device < 0 || device >= ndev) return NLTE_E_INVALID;
    auto* c = new nlte_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    try {
        HIPCHK(hipSetDevice(device));
        upload_constants();
        HIPCHK(scratch_address(device, &c->scratch));
        size_t fr = 0, tot = 0;
        HIPCHK(hipMemGetInfo(&fr, &tot));
        c->budget = hbm_budget ? hbm_budget : size_t(0.9 * double(fr));
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, device));
        c->arch = prop.gcnArchName;
        if (const char* tp = std::getenv("NLTE3D_TUNE_CACHE")) {
            c->tune_path = tp;
            const std::string pre = c->arch + "|";
            for (const auto& kv : read_tune_file(c->tune_path))
                if (kv.first.compare(0, pre.size(), pre) == 0) c->tile_cache[kv.first.substr(pre.size())] = kv.second;
        }
    } catch (const Error& e) {
        delete c;
        return e.code;
    }
    *out = c;
    return NLTE_OK;
}

void nlte_ctx_destroy(nlte_ctx* ctx) {
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->qmu);
        ctx->stopping = true;
        ctx->queue.clear();
    }
    ctx->qcv.notify_all();
    for (auto& t : ctx->workers) t.join();
    ctx->workers.clear();
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (auto& kv : ctx->jobs) delete kv.second;
        ctx->jobs.clear();
    }
    delete ctx;
}

const char* nlte_last_error(const nlte_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

nlte_status nlte_atom_create(nlte_ctx* ctx, const nlte_atom_desc* d, nlte_atom** out) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(d && out, "null argument");
        REQUIRE(d->nlevel >= 2 && d->nlevel <= kMaxLevels, "nlevel must be 2..8");
        REQUIRE(d->nline >= 1 && d->nline <= kMaxLines, "nline must be 1..16");
        REQUIRE(d->ncont >= 0 && d->ncont <= kMaxLevels, "ncont must be 0..8");
        REQUIRE(d->ncoll >= 0 && d->ncoll <= kMaxLevels * kMaxLevels, "too many collision entries");
        REQUIRE(d->mass_amu > 0 && d->xi >= 0, "mass must be > 0 and xi >= 0");
        auto a = std::make_unique<nlte_atom>();
        AtomInfo& I = a->info;
        I.N = d->nlevel;
        I.nline = d->nline;
        I.ncont = d->ncont;
        I.ncoll = d->ncoll;
        I.mass = d->mass_amu;
        I.xi = d->xi;
        I.eps = d->epsilon;
        I.eps_mode = d->epsilon > 0 ? 1 : 0;
        REQUIRE(!I.eps_mode || d->epsilon < 1.0, "epsilon must be < 1");
        for (int i = 0; i < I.N; ++i) {
            REQUIRE(d->levels[i].g > 0 && std::isfinite(d->levels[i].E), "bad level data");
            I.E[i] = d->levels[i].E;
            I.g[i] = d->levels[i].g;
            I.stage[i] = d->levels[i].stage;
        }
        int fs = 0;
        for (int l = 0; l < I.nline; ++l) {
            const nlte_line_desc& s = d->lines[l];
            LineInfo& ln = I.line[l];
            REQUIRE(s.lower >= 0 && s.upper < I.N && s.lower != s.upper, "bad line level indices");
            REQUIRE(I.E[s.upper] > I.E[s.lower], "line upper level must lie above the lower");
            REQUIRE(s.A > 0 && s.nfreq >= 2 && s.q, "line needs A > 0 and >= 2 frequencies");
            for (int m = 1; m < s.nfreq; ++m) REQUIRE(s.q[m] > s.q[m - 1], "line frequencies must increase");
            ln.lower = s.lower; ln.upper = s.upper; ln.fstart = fs; ln.nfreq = s.nfreq;
            ln.gauss = (s.gamma_rad == 0.0 && s.gamma_vdw == 0.0) ? 1 : 0;
            ln.nu0 = kC * (I.E[s.upper] - I.E[s.lower]);
            ln.A = s.A;
            ln.Bji = s.A * kC * kC / (2.0 * kH * ln.nu0 * ln.nu0 * ln.nu0);
            ln.Bij = I.g[s.upper] / I.g[s.lower] * ln.Bji;
            ln.hnu4pi = kH * ln.nu0 / (4.0 * kPI);
            ln.gamma_rad = s.gamma_rad;
            ln.gamma_vdw = s.gamma_vdw;
            // trapezoid weights in Hz on nu = nu0 (1 + q/c)
            for (int m = 0; m < s.nfreq; ++m) {
                double w = 0.0;
                if (m > 0) w += 0.5 * (s.q[m] - s.q[m - 1]);
                if (m + 1 < s.nfreq) w += 0.5 * (s.q[m + 1] - s.q[m]);
                a->q.push_back(s.q[m]);
                a->wnu.push_back(w * ln.nu0 / kC);
                a->line_of.push_back(l);
            }
            fs += s.nfreq;
        }
        a->nf = fs;
        for (int c = 0; c < I.ncont; ++c) {
            const nlte_cont_desc& s = d->continua[c];
            REQUIRE(s.lower >= 0 && s.upper < I.N && I.stage[s.upper] == I.stage[s.lower] + 1,
                    "continuum must link stage s to stage s+1");
            I.cont_lower[c] = s.lower; I.cont_upper[c] = s.upper; I.cont_alpha0[c] = s.alpha0;
        }
        I.cont_active = 0;
        if (d->ncont_nu > 0) {
            REQUIRE(d->cont_nu && I.ncont >= 1, "active continua need a frequency grid and continua");
            const int nfc = d->ncont_nu;
            for (int k = 0; k < nfc; ++k)
                REQUIRE(std::isfinite(d->cont_nu[k]) && d->cont_nu[k] > 0 && (k == 0 || d->cont_nu[k] > d->cont_nu[k - 1]),
                        "continuum frequencies must be positive and increasing");
            a->cnu.assign(d->cont_nu, d->cont_nu + nfc);
            a->ce.resize(nfc);
            for (int k = 0; k < nfc; ++k) a->ce[k] = 2.0 * kH * a->cnu[k] * a->cnu[k] * a->cnu[k] / (kC * kC);
            a->calpha.assign(size_t(I.ncont) * nfc, 0.0);
            a->cfw.assign(size_t(I.ncont) * nfc, 0.0);
            // the distinct upper levels, in order of first appearance
            I.cont_nup = 0;
            for (int c = 0; c < I.ncont; ++c) {
                int u = 0;
                while (u < I.cont_nup && I.cont_ulev[u] != I.cont_upper[c]) ++u;
                if (u == I.cont_nup) {
                    REQUIRE(I.cont_nup < kMaxContUp, "active continua may end on at most 4 upper levels");
                    I.cont_ulev[I.cont_nup++] = I.cont_upper[c];
                }
                I.cont_uidx[c] = u;
            }
            // the line sweeps carry no bound-free opacity: every line must lie below every edge
            double edge = HUGE_VAL;
            for (int c = 0; c < I.ncont; ++c) edge = std::min(edge, kC * (I.E[I.cont_upper[c]] - I.E[I.cont_lower[c]]));
            for (int l = 0; l < I.nline; ++l) {
                const nlte_line_desc& s = d->lines[l];
                REQUIRE(I.line[l].nu0 * (1.0 + s.q[s.nfreq - 1] / kC) < edge,
                        "with active continua every line frequency must lie below every continuum edge");
            }
            for (int c = 0; c < I.ncont; ++c) {
                const double nue = kC * (I.E[I.cont_upper[c]] - I.E[I.cont_lower[c]]);
                int k0 = 0;
                while (k0 < nfc && a->cnu[k0] < nue * (1.0 - 1e-12)) ++k0;
                REQUIRE(k0 < nfc && std::fabs(a->cnu[k0] / nue - 1.0) < 1e-9,
                        "the continuum frequency grid must contain every edge");
                for (int k = k0; k < nfc; ++k) {
                    const double r = nue / a->cnu[k];
                    a->calpha[size_t(c) * nfc + k] = I.cont_alpha0[c] * r * r * r;
                    double w = 0.0;
                    if (k > k0) w += 0.5 * (a->cnu[k] - a->cnu[k - 1]);
                    if (k + 1 < nfc) w += 0.5 * (a->cnu[k + 1] - a->cnu[k]);
                    a->cfw[size_t(c) * nfc + k] = 4.0 * kPI * w / (kH * a->cnu[k]);
                }
            }
            I.cont_active = 1;
        }
        for (int c = 0; c < I.ncoll; ++c) {
            const nlte_coll_desc& s = d->collisions[c];
            REQUIRE(s.lower >= 0 && s.upper < I.N && s.lower != s.upper && s.T_ref > 0, "bad collision entry");
            I.coll_lower[c] = s.lower; I.coll_upper[c] = s.upper;
            I.coll_cul[c] = s.c_ul; I.coll_Tref[c] = s.T_ref; I.coll_beta[c] = s.beta;
        }
        *out = a.release();
        return NLTE_OK;
    });
}

void nlte_atom_destroy(nlte_ctx*, nlte_atom* atom) { delete atom; }

nlte_status nlte_atmos_create(nlte_ctx* ctx, const nlte_atmos_desc* d, nlte_atmos** out) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(d && out && d->z, "null argument");
        REQUIRE(d->nx >= 1 && d->ny >= 1 && d->nz >= 2, "grid must be at least 1x1x2");
        // sweep cells are addressed by 32-bit byte offsets within a plane row
        REQUIRE(double(d->nx) * d->ny * 24.0 < 4294967296.0, "nx*ny must stay below 178,956,970");
        REQUIRE(d->dx > 0 && d->dy > 0, "spacings must be positive");
        for (int k = 1; k < d->nz; ++k) REQUIRE(d->z[k] > d->z[k - 1], "z must increase strictly");
        REQUIRE(d->T && d->ne && d->nH && d->ntot && d->vx && d->vy && d->vz, "missing atmosphere field");
        auto a = std::make_unique<nlte_atmos>();
        a->nx = d->nx; a->ny = d->ny; a->nz = d->nz; a->dx = d->dx; a->dy = d->dy;
        a->z.assign(d->z, d->z + d->nz);
        const size_t nv = size_t(d->nx) * d->ny * d->nz;
        const int nchi = d->chi_c ? d->nchi : 0;
        REQUIRE(nchi >= 0 && nchi <= kMaxLines, "nchi must be 0..16");
        a->nline_chic = nchi;
        const double* fields[7] = {d->T, d->ne, d->nH, d->ntot, d->vx, d->vy, d->vz};
        if (d->mem_kind == NLTE_MEM_HOST) {
            for (int q = 0; q < 7; ++q) REQUIRE(finite_host(fields[q], nv), "non-finite atmosphere value");
            if (nchi) REQUIRE(finite_host(d->chi_c, nv * nchi), "non-finite background opacity");
            for (size_t i = 0; i < nv; ++i) {
                REQUIRE(d->T[i] > 0, "temperature must be positive");
                REQUIRE(d->ne[i] >= 0 && d->nH[i] >= 0 && d->ntot[i] > 0, "densities must be non-negative, ntot > 0");
            }
            for (size_t i = 0; i < nv * nchi; ++i) REQUIRE(d->chi_c[i] >= 0, "background opacity must be >= 0");
        }
        a->prim.alloc(ctx, sizeof(double) * (7 + nchi) * nv);
        const hipMemcpyKind kd = d->mem_kind == NLTE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        for (int q = 0; q < 7; ++q)
            HIPCHK(hipMemcpyAsync(a->prim.as<double>() + size_t(q) * nv, fields[q], sizeof(double) * nv, kd, ctx->stream));
        if (nchi)
            HIPCHK(hipMemcpyAsync(a->prim.as<double>() + size_t(7) * nv, d->chi_c, sizeof(double) * nv * nchi, kd, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        *out = a.release();
        return NLTE_OK;
    });
}

void nlte_atmos_destroy(nlte_ctx* ctx, nlte_atmos* atmos) {
    if (!atmos) return;
    if (ctx) {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        delete atmos;
        return;
    }
    delete atmos;
}

}  // extern "C"

static bool transfer_ops_ok(const nlte_params* p) {
    auto ok = [](int op) { return op == NLTE_RESTRICT_FULL || op == NLTE_RESTRICT_HALF || op == NLTE_RESTRICT_INJECT; };
    return ok(p->restriction) && ok(p->coarse_atmos) &&
           (p->interpolation == NLTE_INTERP_TRILINEAR || p->interpolation == NLTE_INTERP_HERMITE) &&
           (p->sc_interp == NLTE_SC_BILINEAR || p->sc_interp == NLTE_SC_HERMITE);
}

// Checks of the solve parameters shared by nlte_job_create and nlte_submit.
static void check_params(const nlte_params* p, const nlte_atom* atom) {
    REQUIRE(!(atom->info.cont_active && p->sc_interp == NLTE_SC_HERMITE),
            "active continua are swept with bilinear upwind interpolation only");
    REQUIRE(p->method >= NLTE_MALI && p->method <= NLTE_FMG, "unknown method");
    REQUIRE(p->precision == NLTE_FP64 || p->precision == NLTE_MIXED, "unknown precision");
    REQUIRE(transfer_ops_ok(p), "unknown restriction or interpolation scheme");
    REQUIRE(p->nu0 >= 0 && p->nu1 >= 0 && p->nu2 >= 0 && p->nu3 >= 0 && p->nu_fmg >= 0,
            "iteration counts must be >= 0");
    REQUIRE(p->repair_frac > 0 && p->repair_frac < 1, "repair_frac must lie in (0, 1)");
    REQUIRE(p->max_iter >= 0, "max_iter must be >= 0");
    REQUIRE(p->init >= NLTE_INIT_ZERO_RAD && p->init <= NLTE_INIT_USER, "unknown initialisation");
    REQUIRE(std::isfinite(p->diverge_growth) && p->diverge_growth >= 0, "diverge_growth must be >= 0");
    REQUIRE(p->sweep_kernel == NLTE_SWEEP_AUTO || p->sweep_kernel == NLTE_SWEEP_PLANE_STEP, "unknown sweep kernel");
    REQUIRE(p->dirs_per_block == 0 || p->dirs_per_block == 3 || p->dirs_per_block == 6 || p->dirs_per_block == 12,
            "dirs_per_block must be 0, 3, 6 or 12");
}

extern "C" {

nlte_status nlte_job_create(nlte_ctx* ctx, const nlte_atmos* atmos, const nlte_atom* atom,
                            const nlte_params* params, nlte_job* job) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(atmos && atom && params && job, "null argument");
        check_params(params, atom);
        std::unique_ptr<JobBase> j;
        if (params->precision == NLTE_FP64) {
            auto* p = new Job<double>(ctx);
            j.reset(p);
            p->prec = NLTE_FP64;
            p->build(atmos, atom, params);
        } else {
            auto* p = new Job<float>(ctx);
            j.reset(p);
            p->prec = NLTE_MIXED;
            p->build(atmos, atom, params);
        }
        const int64_t id = ctx->next_job++;
        ctx->jobs[id] = j.release();
        *job = id;
        return NLTE_OK;
    });
}

nlte_status nlte_job_run(nlte_ctx* ctx, nlte_job job, nlte_result* result) {
    return guarded(ctx, [&]() -> nlte_status {
        JobBase* j = find_job(ctx, job);
        nlte_result r{};
        j->run(&r);
        if (result) *result = r;
        return r.status;
    });
}

nlte_status nlte_solve(nlte_ctx* ctx, const nlte_atmos* atmos, const nlte_atom* atom, const nlte_params* params,
                       nlte_result* result, nlte_job* job) {
    nlte_job id = 0;
    nlte_status s = nlte_job_create(ctx, atmos, atom, params, &id);
    if (s < 0) return s;
    s = nlte_job_run(ctx, id, result);
    if (s < 0) {
        std::string msg = ctx->err;
        nlte_release(ctx, id);
        ctx->err = msg;
        return s;
    }
    if (job) *job = id;
    else nlte_release(ctx, id);
    return s;
}

nlte_status nlte_release(nlte_ctx* ctx, nlte_job job) {
    return guarded(ctx, [&]() -> nlte_status {
        JobBase* j = find_job(ctx, job, false);
        if (j->served) {
            std::unique_lock<std::mutex> lk(ctx->qmu);
            auto it = std::find(ctx->queue.begin(), ctx->queue.end(), j);
            if (it != ctx->queue.end()) ctx->queue.erase(it);
            else   // admitted: wait for its worker to publish the final state
                ctx->qcv.wait(lk, [&]() { return j->state >= NLTE_JOB_DONE; });
        } else {
            HIPCHK(hipStreamSynchronize(ctx->stream));
        }
        delete j;
        ctx->jobs.erase(job);
        ctx->qcv.notify_all();               // freed memory may admit a queued job
        return NLTE_OK;
    });
}

nlte_status nlte_get_populations(nlte_ctx* ctx, nlte_job job, int level, double* dst, int dst_mem) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(dst, "null destination");
        find_job(ctx, job)->get_pops(level, dst, dst_mem);
        return NLTE_OK;
    });
}

nlte_status nlte_set_populations(nlte_ctx* ctx, nlte_job job, int level, const double* src, int src_mem) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(src, "null source");
        find_job(ctx, job)->set_pops(level, src, src_mem);
        return NLTE_OK;
    });
}

nlte_status nlte_get_source_function(nlte_ctx* ctx, nlte_job job, double* dst, int dst_mem) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(dst, "null destination");
        find_job(ctx, job)->source_function(dst, dst_mem);
        return NLTE_OK;
    });
}

nlte_status nlte_emergent_intensity(nlte_ctx* ctx, nlte_job job, int ndir, const double* mu, float* dst,
                                    int dst_mem) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(ndir >= 1 && mu && dst, "bad emergent-intensity arguments");
        find_job(ctx, job)->emergent(ndir, mu, dst, dst_mem);
        return NLTE_OK;
    });
}

nlte_status nlte_emergent_continuum_intensity(nlte_ctx* ctx, nlte_job job, int ndir, const double* mu, float* dst,
                                              int dst_mem) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(ndir >= 1 && mu && dst, "bad emergent-intensity arguments");
        find_job(ctx, job)->emergent_continuum(ndir, mu, dst, dst_mem);
        return NLTE_OK;
    });
}

nlte_status nlte_emergent_intensity_noalloc(nlte_ctx* ctx, nlte_job job, int ndir, const double* mu, float* dst) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(ndir >= 1 && mu && dst, "bad emergent-intensity arguments");
        REQUIRE(device_memory(dst), "the allocation-free emergent intensity writes device memory only");
        REQUIRE(ctx->scratch, "no scratch address for this device");
        find_job(ctx, job)->emergent_into(ndir, mu, dst, static_cast<double*>(ctx->scratch), kScratchBytes);
        return NLTE_OK;
    });
}

nlte_status nlte_batch_run(nlte_ctx* ctx, int njobs, const nlte_job* jobs, nlte_result* results) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(njobs >= 1 && jobs && results, "bad batch arguments");
        std::vector<JobBase*> js;
        for (int i = 0; i < njobs; ++i) {
            JobBase* j = find_job(ctx, jobs[i]);
            REQUIRE(!j->served, "served jobs are batched by the serving loop");
            REQUIRE(std::find(js.begin(), js.end(), j) == js.end(), "a job appears twice in the batch");
            js.push_back(j);
        }
        std::string msg;
        const nlte_status s = js[0]->prec == NLTE_FP64 ? run_batch<double>(ctx, js, ctx->stream, results, &msg)
                                                       : run_batch<float>(ctx, js, ctx->stream, results, &msg);
        if (s < 0) throw Error(s, msg);
        nlte_status warn = NLTE_OK;
        for (int i = 0; i < njobs; ++i) warn = std::max(warn, results[i].status);
        return warn;
    });
}

nlte_status nlte_job_stats(nlte_ctx* ctx, nlte_job job, nlte_result* out) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(out, "null result");
        find_job(ctx, job)->stats(out);
        return NLTE_OK;
    });
}

int nlte_history(nlte_ctx* ctx, nlte_job job, double* C, int cap) {
    if (!ctx) return -1;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->jobs.find(job);
    if (it == ctx->jobs.end()) return -1;
    const auto& h = it->second->history;
    const int n = int(h.size());
    for (int i = 0; i < n && i < cap && C; ++i) C[i] = h[i];
    return n;
}

nlte_status nlte_formal_solution(nlte_ctx* ctx, nlte_job job, int level, void* jeff, void* oml, int dst_mem) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(jeff && oml, "null destination");
        find_job(ctx, job)->formal_solution_out(level, jeff, oml, dst_mem);
        return NLTE_OK;
    });
}

nlte_status nlte_mali(nlte_ctx* ctx, nlte_job job, int level, int iters, double* C_out) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(iters >= 0, "iters must be >= 0");
        const double c = find_job(ctx, job)->mali_hook(level, iters);
        if (C_out) *C_out = c;
        return NLTE_OK;
    });
}

nlte_status nlte_rate_solve(nlte_ctx* ctx, nlte_job job, int level, const void* jeff, const void* oml, int src_mem,
                            double* C_out) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(jeff && oml, "null radiation input");
        REQUIRE(src_mem == NLTE_MEM_HOST || src_mem == NLTE_MEM_DEVICE, "bad memory kind");
        const double c = find_job(ctx, job)->rate_solve_hook(level, jeff, oml, src_mem);
        if (C_out) *C_out = c;
        return NLTE_OK;
    });
}

nlte_status nlte_residual(nlte_ctx* ctx, nlte_job job, int level, double* dst, int dst_mem) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(dst, "null destination");
        find_job(ctx, job)->residual_out(level, dst, dst_mem);
        return NLTE_OK;
    });
}

nlte_status nlte_vcycle(nlte_ctx* ctx, nlte_job job, int level, int first, long long* repairs) {
    return guarded(ctx, [&]() -> nlte_status {
        JobBase* j = find_job(ctx, job);
        j->vcycle_hook(level, first);
        if (repairs) *repairs = j->repair_count();
        return NLTE_OK;
    });
}

nlte_status nlte_restrict(nlte_ctx* ctx, nlte_job job, int level, int nq, const double* src, double* dst) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(nq >= 1 && src && dst, "bad restriction arguments");
        REQUIRE(device_memory(src) && device_memory(dst), "restriction arrays must be device memory");
        find_job(ctx, job)->restrict_hook(level, nq, src, dst);
        return NLTE_OK;
    });
}

nlte_status nlte_prolong(nlte_ctx* ctx, nlte_job job, int level, int nq, const double* src, double* dst) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(nq >= 1 && src && dst, "bad prolongation arguments");
        REQUIRE(device_memory(src) && device_memory(dst), "prolongation arrays must be device memory");
        find_job(ctx, job)->prolong_hook(level, nq, src, dst);
        return NLTE_OK;
    });
}

nlte_status nlte_voigt(nlte_ctx* ctx, int precision, int n, const double* a, const double* u, double* H) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(precision == NLTE_FP64 || precision == NLTE_MIXED, "precision must be NLTE_FP64 or NLTE_MIXED");
        REQUIRE(n >= 0 && (n == 0 || (a && u && H)), "bad Voigt arguments");
        if (n == 0) return NLTE_OK;
        REQUIRE(device_memory(a) && device_memory(u) && device_memory(H), "Voigt arrays must be device memory");
        if (precision == NLTE_FP64)
            voigt_eval_kernel<double><<<blocks_for(size_t(n), 256), 256, 0, ctx->stream>>>(a, u, H, n);
        else
            voigt_eval_kernel<float><<<blocks_for(size_t(n), 256), 256, 0, ctx->stream>>>(a, u, H, n);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return NLTE_OK;
    });
}

}  // extern "C"

extern "C" {

nlte_status nlte_serve_batching(nlte_ctx* ctx, int batch_max) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(batch_max >= 1 && batch_max <= 64, "batch_max must be 1..64");
        std::lock_guard<std::mutex> lk(ctx->qmu);
        ctx->batch_max = batch_max;
        return NLTE_OK;
    });
}

nlte_status nlte_serve_config(nlte_ctx* ctx, int max_running) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(max_running >= 1 && max_running <= 16, "max_running must be 1..16");
        std::lock_guard<std::mutex> lk(ctx->qmu);
        while (int(ctx->workers.size()) < max_running) ctx->workers.emplace_back(serve_worker, ctx);
        ctx->max_running = int(ctx->workers.size());
        return NLTE_OK;
    });
}

nlte_status nlte_estimate_footprint(nlte_ctx* ctx, const nlte_atmos* atmos, const nlte_atom* atom,
                                    const nlte_params* params, size_t* bytes) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(atmos && atom && params && bytes, "null argument");
        *bytes = job_footprint(ctx, atmos, atom, params);
        return NLTE_OK;
    });
}

nlte_status nlte_submit(nlte_ctx* ctx, const nlte_atmos* atmos, const nlte_atom* atom, const nlte_params* params,
                        nlte_job* job) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(atmos && atom && params && job, "null argument");
        check_params(params, atom);
        REQUIRE(params->init != NLTE_INIT_USER && params->top_I == nullptr,
                "served jobs take no host arrays in params");
        const int nlev = std::max(1, params->method == NLTE_MALI ? 1 : params->nlev);
        const int step = 1 << (nlev - 1);
        REQUIRE(atmos->nx % step == 0 && atmos->ny % step == 0 && (atmos->nz - 1) % step == 0,
                "grid does not admit the requested number of levels");
        if (ctx->workers.empty()) {
            std::lock_guard<std::mutex> lk(ctx->qmu);
            ctx->workers.emplace_back(serve_worker, ctx);
            ctx->max_running = 1;
        }
        std::unique_ptr<JobBase> j;
        if (params->precision == NLTE_FP64) j.reset(new Job<double>(ctx));
        else j.reset(new Job<float>(ctx));
        j->prec = params->precision;
        j->params = *params;
        j->served = true;
        j->src_atmos = atmos;
        j->src_atom = atom;
        j->footprint = job_footprint(ctx, atmos, atom, params);
        REQUIRE(j->footprint <= ctx->budget, "job footprint exceeds the context's HBM budget");
        j->state = 0;
        j->t_submit = now_s();
        const int64_t id = ctx->next_job++;
        JobBase* raw = j.release();
        ctx->jobs[id] = raw;
        {
            std::lock_guard<std::mutex> lk(ctx->qmu);
            ctx->queue.push_back(raw);
        }
        ctx->qcv.notify_all();
        *job = id;
        return NLTE_W_QUEUED;
    });
}

nlte_status nlte_poll(nlte_ctx* ctx, nlte_job job, int* state) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(state, "null state");
        *state = find_job(ctx, job, false)->state;
        return NLTE_OK;
    });
}

nlte_status nlte_wait(nlte_ctx* ctx, nlte_job job, int timeout_ms) {
    if (!ctx) return NLTE_E_INVALID;
    JobBase* j = nullptr;
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        auto it = ctx->jobs.find(job);
        if (it == ctx->jobs.end()) return NLTE_E_INVALID;
        j = it->second;
    }
    const double t0 = now_s();
    std::unique_lock<std::mutex> lk(ctx->qmu);
    while (j->state < 2) {
        if (timeout_ms >= 0 && (now_s() - t0) * 1e3 >= timeout_ms) return NLTE_W_QUEUED;
        ctx->qcv.wait_for(lk, std::chrono::milliseconds(2));
    }
    return j->final_status;
}

nlte_status nlte_job_info(nlte_ctx* ctx, nlte_job job, nlte_job_info_t* info) {
    return guarded(ctx, [&]() -> nlte_status {
        REQUIRE(info, "null info");
        JobBase* j = find_job(ctx, job, false);
        std::memset(info, 0, sizeof(*info));
        info->state = j->state;
        info->status = j->final_status;
        info->t_submit = j->t_submit;
        info->t_admit = j->t_admit;
        info->t_done = j->t_done;
        info->footprint = j->footprint;
        info->batch = j->batch_id;
        if (j->state >= 2) info->result = j->res;
        std::snprintf(info->error, sizeof(info->error), "%s", j->error.c_str());
        return NLTE_OK;
    });
}

}  // extern "C"
