// libigr host runtime: context, scratch, boundary tables, launch sequences
// and the C ABI declared in include/igr.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "igr.h"
#include "igr_flux.h"
#include "igr_sigma.h"
#include "igr_adjoint.h"
#include "igr_kernels.h"
#include "igr_viscous.h"

using namespace igr;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define IGR_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? IGR_ENOMEM : IGR_EHIP,                         \
                        std::string(#call) + ": " + hipGetErrorString(e_));                        \
    } while (0)

#define IGR_TRY(expr)              \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != IGR_OK) return rc_; \
    } while (0)

enum KernelId {
    K_BC_STATE, K_BC_SIGMA, K_SOURCE, K_JACOBI, K_FLUX, K_DT,
    K_SUMS,     K_RESID,    K_SWEEP,  K_ADJOINT, K_VISCOUS, K_STRESS, K_COUNT
};
const char* const kKernelNames[K_COUNT] = {"bc_state", "bc_sigma", "source",  "jacobi", "flux_rk", "dt",
                                           "sums",     "resid",    "sweep",   "adjoint", "viscous", "stress"};

struct TimingRecord {
    int kernel;
    hipEvent_t start, stop;
};

}  // namespace

struct igr_ctx {
    Geom g{};
    int nx = 0, ny = 0, nz = 0;
    double dx = 0, dy = 0, dz = 0;
    int precision = IGR_F64;
    int nsweeps = 5;
    int order = 5;         // reconstruction order (5 or 3)
    int smoother = IGR_SMOOTH_JACOBI;
    double mu = 0.0, zeta = 0.0;   // shear and bulk viscosity (eq. (5))
    bool viscous = false;          // mu or zeta nonzero
    int sigma_block = 1;   // Sigma pass structure (1: single sweeps, 2: first + two-sweep passes, 3..5: fused march)
    int faces[6] = {0, 0, 0, 0, 0, 0};
    int device = 0;
    size_t esize = 8;     // storage bytes per element of a state (U^n, rhs)
    size_t dsize = 8;     // storage bytes per element of an RK stage buffer
    size_t ssize = 8;     // storage bytes per element of Sigma
    size_t csize = 8;     // arithmetic bytes per element (source array, stored 1/rho)
    std::vector<igr_patch> patches;
    std::vector<int> h_owner;     // per x-min column (k*ny + j): nearest disc or -1
    int* d_owner = nullptr;
    double* d_chi = nullptr;
    double* d_jet = nullptr;
    void* d_Ua = nullptr;
    void* d_Ub = nullptr;
    void* d_sig2 = nullptr;
    void* d_b = nullptr;
    void* d_ir = nullptr;         // 1/rho written by the first sweep (split form)
    void* d_Unb = nullptr;        // split form: the other FP32 state of the U^n / U^(n+1) ping-pong
    double* d_jet0 = nullptr;     // split form: zero jet states (ghosts of the stage differences)
    void* d_G = nullptr;          // viscous: the 6 stress components (arithmetic type)
    double* d_partial = nullptr;
    double* d_scalars = nullptr;  // [0] dt, [1..5] sums, [6] residual
    double* d_speed = nullptr;    // per-flux-block CFL maxima left by a step's last stage
    int* d_flag = nullptr;
    bool timing = false;
    std::vector<TimingRecord> records;
    std::vector<hipEvent_t> event_pool;
    double kernel_ms[K_COUNT] = {};
    long long kernel_count[K_COUNT] = {};
    // adjoint scratch (FP64, allocated on first adjoint call)
    int adj_sweeps = -1;
    std::vector<double*> adj;     // see adjoint_buffers()
};

namespace {

size_t field_bytes(const igr_ctx* c, size_t elem) { return (size_t)c->g.fs * elem; }

hipEvent_t pooled_event(igr_ctx* c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch helper: records start/stop events around the launch when timing.
template <class F>
int launch(igr_ctx* c, int kernel, hipStream_t s, F&& fn) {
    TimingRecord rec{kernel, nullptr, nullptr};
    if (c->timing) {
        rec.start = pooled_event(c);
        rec.stop = pooled_event(c);
    }
    // a launch whose events cannot be recorded is simply not timed
    bool timed = rec.start && rec.stop && hipEventRecord(rec.start, s) == hipSuccess;
    fn();
    hipError_t e = hipGetLastError();
    timed = timed && e == hipSuccess && hipEventRecord(rec.stop, s) == hipSuccess;
    if (timed) {
        c->records.push_back(rec);
    } else {   // unused events go back to the pool
        if (rec.start) c->event_pool.push_back(rec.start);
        if (rec.stop) c->event_pool.push_back(rec.stop);
    }
    if (e != hipSuccess) return fail(IGR_EHIP, std::string("launch of ") + kKernelNames[kernel] + ": " + hipGetErrorString(e));
    return IGR_OK;
}

// Folds the recorded launch times into the per-kernel totals.  The records
// leave the context first, and every record's two events go back to the
// pool exactly once, also when a query fails part way (the failed record
// and the ones after it are then dropped untimed).
int collect_timing(igr_ctx* c) {
    std::vector<TimingRecord> recs;
    recs.swap(c->records);
    hipError_t err = hipSuccess;
    const char* what = "";
    for (const TimingRecord& r : recs) {
        if (err == hipSuccess) {
            float ms = 0.f;
            err = hipEventSynchronize(r.stop);
            what = "hipEventSynchronize";
            if (err == hipSuccess) {
                err = hipEventElapsedTime(&ms, r.start, r.stop);
                what = "hipEventElapsedTime";
            }
            if (err == hipSuccess) {
                c->kernel_ms[r.kernel] += ms;
                c->kernel_count[r.kernel] += 1;
            }
        }
        c->event_pool.push_back(r.start);
        c->event_pool.push_back(r.stop);
    }
    if (err != hipSuccess) return fail(IGR_EHIP, std::string(what) + ": " + hipGetErrorString(err));
    return IGR_OK;
}

dim3 cell_block() { return dim3(64, 4, 1); }
dim3 cell_grid(const Geom& g) { return dim3((g.n[0] + 63) / 64, (g.n[1] + 3) / 4, g.n[2]); }

// delta: U holds a split-form stage difference from U^n, whose ghost cells
// were filled already: an inflow ghost of the stage state is
// chi U_jet + (1 - chi)(U^n_ext + delta_ext), so its difference is
// (1 - chi) delta_ext, the same blend with a zero jet state.
template <class T>
int fill_state_ghosts(igr_ctx* c, T* U, hipStream_t s, bool delta = false) {
    const long long tot = bc_face_threads(c->g);
    if (tot / 256 + 1 > 0x7fffffffLL) return fail(IGR_EINVAL, "grid too large for the ghost fill");
    const int blocks = int((tot + 255) / 256);
    const int* owner = c->patches.empty() ? nullptr : c->d_owner;
    const double* jet = delta ? c->d_jet0 : c->d_jet;
    IGR_TRY(launch(c, K_BC_STATE, s, [&] { k_bc_state<T><<<blocks, 256, 0, s>>>(U, c->g, owner, c->d_chi, jet); }));
    return IGR_OK;
}

template <class T>
int fill_sigma_ghosts(igr_ctx* c, T* Sg, hipStream_t s) {
    const long long tot = bc_face_threads(c->g);
    const int blocks = int((tot + 255) / 256);
    IGR_TRY(launch(c, K_BC_SIGMA, s, [&] { k_bc_sigma<T><<<blocks, 256, 0, s>>>(Sg, c->g); }));
    return IGR_OK;
}

// Sigma passes: `nsweeps` Jacobi sweeps split into passes of at most
// SigShape<T>::KMAX levels of the temporally blocked kernel (each pass
// reads rho, m and Sigma once and forms the source itself).  FP64 uses a
// shorter tile (fewer threads per block, more registers per thread).
#ifndef IGR_SIG_KMAX_F64
#define IGR_SIG_KMAX_F64 3
#endif
#ifndef IGR_SIG_NR_F64
#define IGR_SIG_NR_F64 12
#endif
#ifndef IGR_SIG_KMAX_F32
#define IGR_SIG_KMAX_F32 5
#endif
#ifndef IGR_SIG_NR_F32
#define IGR_SIG_NR_F32 16
#endif
template <class T>
struct SigShape {
    static constexpr int KMAX = IGR_SIG_KMAX_F32;
    static constexpr int NR = IGR_SIG_NR_F32;
};
template <>
struct SigShape<double> {
    static constexpr int KMAX = IGR_SIG_KMAX_F64;
    static constexpr int NR = IGR_SIG_NR_F64;
};

template <class T, int K>
int sigma_pass(igr_ctx* c, const T* U, const T* Sin, T* Sout, hipStream_t s) {
    constexpr int NR = SigShape<T>::NR;
    constexpr int TXo = SIG_TX - 2 * K, TYo = NR - 2 * K;
    const int tiles_x = (c->g.n[0] + TXo - 1) / TXo;
    const int tiles_y = (c->g.n[1] + TYo - 1) / TYo;
    const long long tiles = (long long)tiles_x * tiles_y;
    long long zc = (tiles * c->g.n[2] + 1023) / 1024;   // aim at >= ~1024 blocks
    if (zc < 16) zc = 16;
    if (zc > 128) zc = 128;
    if (zc > c->g.n[2]) zc = c->g.n[2];
    const long long chunks = (c->g.n[2] + zc - 1) / zc;
    const long long blocks = tiles * chunks;
    if (blocks > 0x7fffffffLL) return fail(IGR_EINVAL, "grid too large for the Sigma launch");
    return launch(c, K_JACOBI, s, [&] {
        k_sigma_march<T, K, NR><<<dim3(unsigned(blocks)), dim3(SIG_TX, NR), 0, s>>>(U, Sin, Sout, c->g, tiles_x,
                                                                                  tiles_y, int(zc));
    });
}

template <class T>
int sigma_pass_k(igr_ctx* c, int k, const T* U, const T* Sin, T* Sout, hipStream_t s) {
    constexpr int KM = SigShape<T>::KMAX;
    if (k >= 5 && KM >= 5) return sigma_pass<T, (KM >= 5 ? 5 : 1)>(c, U, Sin, Sout, s);
    if (k >= 4 && KM >= 4) return sigma_pass<T, (KM >= 4 ? 4 : 1)>(c, U, Sin, Sout, s);
    if (k >= 3 && KM >= 3) return sigma_pass<T, (KM >= 3 ? 3 : 1)>(c, U, Sin, Sout, s);
    if (k >= 2 && KM >= 2) return sigma_pass<T, (KM >= 2 ? 2 : 1)>(c, U, Sin, Sout, s);
    return sigma_pass<T, 1>(c, U, Sin, Sout, s);
}

// Launch of the two-sweep pass: 64 x (NR-2) output tiles, z chunks sized
// for about IGR_PAIR_BLOCKS blocks of 64 x (NR+1) threads.
// Last-level (Infinity) cache of one MI355X, bytes.
#ifndef IGR_LLC_BYTES
#define IGR_LLC_BYTES (256.0 * 1024 * 1024)
#endif

#ifndef IGR_PAIR_BLOCKS
#define IGR_PAIR_BLOCKS 2048
#endif
#ifndef IGR_PAIR_ZC_MIN
#define IGR_PAIR_ZC_MIN 8
#endif
#ifndef IGR_PAIR_ZC_MAX
#define IGR_PAIR_ZC_MAX 128
#endif
// Launch shape of a two-sweep pass with NR rows per block.
struct PairShape {
    int tiles_x, tiles_y, zc;
    long long blocks;
};
PairShape pair_shape(const Geom& g, int nr) {
    PairShape sh;
    sh.tiles_x = (g.n[0] + 63) / 64;
    sh.tiles_y = (g.n[1] + nr - 3) / (nr - 2);
    const long long tiles = (long long)sh.tiles_x * sh.tiles_y;
    long long zc = (tiles * g.n[2] + IGR_PAIR_BLOCKS - 1) / IGR_PAIR_BLOCKS;
    if (zc < IGR_PAIR_ZC_MIN) zc = IGR_PAIR_ZC_MIN;
    if (zc > IGR_PAIR_ZC_MAX) zc = IGR_PAIR_ZC_MAX;
    if (zc > g.n[2]) zc = g.n[2];
    sh.zc = int(zc);
    sh.blocks = tiles * ((g.n[2] + zc - 1) / zc);
    return sh;
}
// CFL maxima left by a first two-sweep pass that forms them: one per wave.
long long pair_speed_slots(const Geom& g) { return pair_shape(g, PAIR_NR_FIRST).blocks * (PAIR_NR_FIRST + 1); }

// speed (FIRST, FP64 state without a difference; nullable): the pass also
// leaves the CFL maxima of U there.  RB: one red-black sweep per pass
// instead of two Jacobi sweeps.  tau (FIRST; nullable): the pass also
// stores the viscous stress of U there.
template <class F, bool FIRST, bool HASD, bool RB = false>
int pair_pass(igr_ctx* c, const typename F::TB* U, const typename F::TD* D, const typename F::TS* Sin,
              typename F::TS* Sout, hipStream_t s, double* speed = nullptr, typename F::C* tau = nullptr) {
    using C = typename F::C;
    const Geom& g = c->g;
    // rows per block: the first pass that also forms the CFL maxima keeps
    // PAIR_NR_FIRST (its speed slots are sized by it)
    constexpr int NR = FIRST ? pair_nr_first<F, HASD>() : pair_nr_later<F>();
    constexpr bool SPD_OK = FIRST && !HASD && sizeof(C) == 8;
    const bool spd = SPD_OK && speed != nullptr;
    const PairShape sh = pair_shape(g, spd ? PAIR_NR_FIRST : NR);
    if (sh.blocks > 0x7fffffffLL) return fail(IGR_EINVAL, "grid too large for the sweep launch");
    C* b = static_cast<C*>(c->d_b);
    C* ir = static_cast<C*>(c->d_ir);
    return launch(c, K_JACOBI, s, [&] {
        if (spd) {
            if constexpr (SPD_OK) {
                const dim3 grid(unsigned(sh.blocks)), block(64, PAIR_NR_FIRST + 1);
                if (tau)
                    k_sweep_pair<F, PAIR_NR_FIRST, true, false, true, RB, true><<<grid, block, 0, s>>>(
                        U, D, Sin, Sout, b, ir, g, sh.zc, sh.tiles_x, sh.tiles_y, speed, c->d_flag, tau, c->mu,
                        c->zeta);
                else
                    k_sweep_pair<F, PAIR_NR_FIRST, true, false, true, RB><<<grid, block, 0, s>>>(
                        U, D, Sin, Sout, b, ir, g, sh.zc, sh.tiles_x, sh.tiles_y, speed, c->d_flag);
            }
        } else {
            const dim3 grid(unsigned(sh.blocks)), block(64, NR + 1);
            if constexpr (FIRST) {
                if (tau) {
                    k_sweep_pair<F, NR, true, HASD, false, RB, true><<<grid, block, 0, s>>>(
                        U, D, Sin, Sout, b, ir, g, sh.zc, sh.tiles_x, sh.tiles_y, nullptr, nullptr, tau, c->mu,
                        c->zeta);
                    return;
                }
            }
            k_sweep_pair<F, NR, FIRST, HASD, false, RB><<<grid, block, 0, s>>>(U, D, Sin, Sout, b, ir, g, sh.zc,
                                                                             sh.tiles_x, sh.tiles_y);
        }
    });
}

// nsweeps Jacobi sweeps from `sig` (warm start); U ghosts must be filled.
// sigma_block 1: one z-marching sweep per pass, the source (and, in FP64,
// 1/rho) formed in the first pass and stored; 2: two sweeps per pass (for
// an even count the first pass also forms the source, else a single first
// sweep does); 3..5: passes of up to that many levels of the
// temporally blocked kernel that forms the source itself.  The last
// iterate ends in `sig` (device copy after an odd number of passes) and
// its ghosts are filled.
#ifndef IGR_SWEEP_BLOCKS
#define IGR_SWEEP_BLOCKS 2048
#endif
#ifndef IGR_SWEEP_ZC_MIN
#define IGR_SWEEP_ZC_MIN 4
#endif
// Single-sweep launch: 64 x ry column tiles, z chunks sized for about
// IGR_SWEEP_BLOCKS blocks.
struct SweepShape {
    int tiles_x, tiles_y, zc;
    long long blocks;
};
SweepShape sweep_shape(const Geom& g, int ry) {
    SweepShape sh;
    sh.tiles_x = (g.n[0] + 63) / 64;
    sh.tiles_y = (g.n[1] + ry - 1) / ry;
    const long long tiles = (long long)sh.tiles_x * sh.tiles_y;
    long long zc = (tiles * g.n[2] + IGR_SWEEP_BLOCKS - 1) / IGR_SWEEP_BLOCKS;
    if (zc < IGR_SWEEP_ZC_MIN) zc = IGR_SWEEP_ZC_MIN;
    if (zc > 64) zc = 64;
    if (zc > g.n[2]) zc = g.n[2];
    sh.zc = int(zc);
    sh.blocks = tiles * ((g.n[2] + zc - 1) / zc);
    return sh;
}
// CFL maxima left by a first sweep that forms them: one per wave.
long long sweep_speed_slots(const Geom& g) { return sweep_shape(g, SWEEP_RY_FIRST).blocks * SWEEP_RY_FIRST; }

// speed (FP64 contexts, nullable): if the solve starts with a single first
// sweep, that sweep also leaves the CFL maxima of U there and *nspeed is
// their count; otherwise *nspeed is 0.  The state swept from is U (+ D
// with HASD: a split-form stage difference).  tau (nullable): if the solve
// starts with a two-level first pass or a single first sweep, that pass
// also stores the viscous stress of the state there and *tau_done is set;
// otherwise (no sweeps, the fused march) it is cleared.
template <class F, bool HASD = false>
int sigma_solve_buf(igr_ctx* c, const typename F::TB* U, const typename F::TD* D, typename F::TS* in,
                    typename F::TS* other, int nsweeps, typename F::TS** result, hipStream_t s,
                    double* speed = nullptr, int* nspeed = nullptr, typename F::C* tau = nullptr,
                    bool* tau_done = nullptr) {
    using C = typename F::C;
    using TS = typename F::TS;
    if (nspeed) *nspeed = 0;
    if (tau_done) *tau_done = false;
    TS* src = in;
    TS* dst = other;
    auto swap = [&] {
        TS* tmp = src;
        src = dst;
        dst = tmp;
    };
    if (c->sigma_block <= 2 || c->smoother == IGR_SMOOTH_RBGS) {
        const Geom& g = c->g;
        const SweepShape sf = sweep_shape(g, SWEEP_RY_FIRST), sl = sweep_shape(g, SWEEP_RY);
        if (sf.blocks > 0x7fffffffLL || sl.blocks > 0x7fffffffLL)
            return fail(IGR_EINVAL, "grid too large for the sweep launch");
        C* b = static_cast<C*>(c->d_b);
        C* ir = static_cast<C*>(c->d_ir);
        auto single = [&](bool first, int colour = -1) {
            TS* out = colour < 0 ? dst : src;   // red-black half-sweeps work in place
            constexpr bool SPD_OK = sizeof(C) == 8 && !HASD;   // CFL maxima formed in the first sweep: FP64
            const bool spd = SPD_OK && first && speed != nullptr;
            if (spd && nspeed) *nspeed = int(sf.blocks * SWEEP_RY_FIRST);
            if (first && tau && tau_done) *tau_done = true;
            return launch(c, K_JACOBI, s, [&] {
                const dim3 gf(unsigned(sf.blocks)), bf(64, SWEEP_RY_FIRST);
                if (first && spd) {
                    if constexpr (SPD_OK) {
                        if (tau)
                            k_sweep_z<F, true, SWEEP_RY_FIRST, true, false, true><<<gf, bf, 0, s>>>(
                                U, D, src, out, b, ir, g, sf.zc, sf.tiles_x, sf.tiles_y, colour, speed, c->d_flag, tau,
                                c->mu, c->zeta);
                        else
                            k_sweep_z<F, true, SWEEP_RY_FIRST, true><<<gf, bf, 0, s>>>(
                                U, D, src, out, b, ir, g, sf.zc, sf.tiles_x, sf.tiles_y, colour, speed, c->d_flag);
                    }
                } else if (first) {
                    if (tau)
                        k_sweep_z<F, true, SWEEP_RY_FIRST, false, HASD, true><<<gf, bf, 0, s>>>(
                            U, D, src, out, b, ir, g, sf.zc, sf.tiles_x, sf.tiles_y, colour, nullptr, nullptr, tau,
                            c->mu, c->zeta);
                    else
                        k_sweep_z<F, true, SWEEP_RY_FIRST, false, HASD><<<gf, bf, 0, s>>>(
                            U, D, src, out, b, ir, g, sf.zc, sf.tiles_x, sf.tiles_y, colour, nullptr, nullptr);
                } else {
                    k_sweep_z<F, false, SWEEP_RY, false, HASD><<<dim3(unsigned(sl.blocks)), dim3(64, SWEEP_RY), 0, s>>>(
                        U, D, src, out, b, ir, g, sl.zc, sl.tiles_x, sl.tiles_y, colour, nullptr, nullptr);
                }
            });
        };
        if (c->smoother == IGR_SMOOTH_RBGS && c->sigma_block == 2) {
            // red-black Gauss-Seidel, one pass per sweep (both halves; the
            // first pass also forms b and, FP64, the CFL maxima of U)
            for (int it = 0; it < nsweeps; ++it) {
                if (it == 0) {
                    const bool spd = sizeof(C) == 8 && !HASD && speed != nullptr;
                    IGR_TRY((pair_pass<F, true, HASD, true>(c, U, D, src, dst, s, spd ? speed : nullptr, tau)));
                    if (spd && nspeed) *nspeed = int(pair_speed_slots(c->g));
                    if (tau && tau_done) *tau_done = true;
                } else {
                    IGR_TRY((pair_pass<F, false, HASD, true>(c, U, D, src, dst, s)));
                }
                swap();
            }
            *result = src;
            return fill_sigma_ghosts(c, src, s);
        }
        if (c->smoother == IGR_SMOOTH_RBGS) {
            // red-black Gauss-Seidel in place, a launch per half-sweep: red
            // (the first also forms b), then black
            for (int it = 0; it < nsweeps; ++it) {
                IGR_TRY(single(it == 0, 0));
                IGR_TRY(single(false, 1));
            }
            *result = src;
            return fill_sigma_ghosts(c, src, s);
        }
        int left = nsweeps;
#ifndef IGR_FIRST_PAIR
#define IGR_FIRST_PAIR 1
#endif
        if (IGR_FIRST_PAIR && c->sigma_block == 2 && left >= 2 && left % 2 == 0) {
            // an even count: the first two sweeps in one pass that also
            // forms the source, then pairs (an odd count keeps the single
            // first sweep, then pairs: measured faster than first pass +
            // pairs + a single sweep)
            // FP64: the pass also forms the CFL maxima of U when asked
            const bool spd = sizeof(C) == 8 && !HASD && speed != nullptr;
            IGR_TRY((pair_pass<F, true, HASD>(c, U, D, src, dst, s, spd ? speed : nullptr, tau)));
            if (spd && nspeed) *nspeed = int(pair_speed_slots(c->g));
            if (tau && tau_done) *tau_done = true;
            swap();
            left -= 2;
        } else if (left > 0) {
            IGR_TRY(single(true));
            swap();
            --left;
        }
        if (c->sigma_block == 2) {
            for (; left >= 2; left -= 2) {
                IGR_TRY((pair_pass<F, false, HASD>(c, U, D, src, dst, s)));
                swap();
            }
        }
        for (; left > 0; --left) {
            IGR_TRY(single(false));
            swap();
        }
    } else if constexpr (!F::SPLIT) {
        // the fused march reads one storage type (igr_init rejects it for the split form)
        using T = typename F::TB;
        const int kmax = c->sigma_block < SigShape<T>::KMAX ? c->sigma_block : SigShape<T>::KMAX;
        int left = nsweeps;
        while (left > 0) {
            const int k = left < kmax ? left : kmax;
            IGR_TRY(sigma_pass_k<T>(c, k, U, src, dst, s));
            left -= k;
            swap();
        }
    } else {
        return fail(IGR_EUNSUPPORTED, "the fused Sigma march needs a plain storage form");
    }
    *result = src;
    return fill_sigma_ghosts(c, src, s);
}

// As sigma_solve_buf from a state U of the step's type, with the result
// always in `sig`.
template <class F>
int sigma_solve_impl(igr_ctx* c, typename F::TB* U, typename F::TS* sig, int nsweeps, hipStream_t s) {
    using TS = typename F::TS;
    TS* res = nullptr;
    IGR_TRY(sigma_solve_buf<F>(c, U, nullptr, sig, static_cast<TS*>(c->d_sig2), nsweeps, &res, s));
    if (res != sig) IGR_HIP(hipMemcpyAsync(sig, res, field_bytes(c, sizeof(TS)), hipMemcpyDeviceToDevice, s));
    return IGR_OK;
}

// Source b into the scratch array (for the residual diagnostic).
template <class T>
int source_impl(igr_ctx* c, const T* U, hipStream_t s) {
    using C = typename Storage<T>::C;
    C* b = static_cast<C*>(c->d_b);
    return launch(c, K_SOURCE, s, [&] { k_source<T, C><<<cell_grid(c->g), cell_block(), 0, s>>>(U, b, c->g); });
}

// Launch shape of the tiled flux kernel: 64 x TY column tiles, z chunks
// sized for >= ~2048 blocks (256 CUs, several resident blocks each).
// Rows per tile: the block (TY+1 waves) must fill the waves one CU can
// hold at the kernel's register use (FP64: 8 per CU, FP32: 12), so one
// block is resident per CU and a launch runs in rounds of 256 blocks.
// Block-count targets (z chunk = tiles * nz / target, within 8..64
// planes), measured on the 256^3 box: FP64 3072 (0.82 ms per launch;
// 2048: 0.84, 768: 0.95), FP32 arithmetic 768, three full rounds of 32-plane
// chunks (0.38 ms; 1024: 0.43, 2048: 0.41).  From 512^3 up the 64-plane
// cap decides.  TY = 3..5 is 20-75 % slower.
#ifndef IGR_FLUX_TY_F64
#define IGR_FLUX_TY_F64 7
#endif
#ifndef IGR_FLUX_TY_F32
#define IGR_FLUX_TY_F32 11
#endif
#ifndef IGR_FLUX_BLOCKS_F64
#define IGR_FLUX_BLOCKS_F64 3072
#endif
#ifndef IGR_FLUX_BLOCKS_F32
#define IGR_FLUX_BLOCKS_F32 768
#endif
template <class T>
struct FluxShape {
    static constexpr int TY = IGR_FLUX_TY_F32;
    static constexpr int BLOCKS = IGR_FLUX_BLOCKS_F32;
};
template <>
struct FluxShape<double> {
    static constexpr int TY = IGR_FLUX_TY_F64;
    static constexpr int BLOCKS = IGR_FLUX_BLOCKS_F64;
};

// The split form's stages 2 and 3 read each value as a base and a
// difference, which needs more registers than the other FP32-arithmetic
// forms: its own tile height and block target.
#ifndef IGR_FLUX_TY_SPLIT
#define IGR_FLUX_TY_SPLIT 11
#endif
#ifndef IGR_FLUX_BLOCKS_SPLIT
#define IGR_FLUX_BLOCKS_SPLIT 768
#endif
template <class F>
struct FluxShapeOf : FluxShape<typename F::C> {};
template <>
struct FluxShapeOf<Split> {
    static constexpr int TY = IGR_FLUX_TY_SPLIT;
    static constexpr int BLOCKS = IGR_FLUX_BLOCKS_SPLIT;
};

#ifndef IGR_FLUX_ZC_MAX
#define IGR_FLUX_ZC_MAX 64
#endif
struct FluxLaunch {
    int tiles_x, tiles_y, zc, chunks;
    long long blocks() const { return (long long)tiles_x * tiles_y * chunks; }
};

FluxLaunch flux_launch(const Geom& g, int ty, int target_blocks) {
    FluxLaunch L;
    L.tiles_x = (g.n[0] + FLUX_TX - 1) / FLUX_TX;
    L.tiles_y = (g.n[1] + ty - 1) / ty;
    const long long tiles = (long long)L.tiles_x * L.tiles_y;
    // long chunks: every chunk re-reads five planes to prime its z queue
    long long zc = (tiles * g.n[2] + target_blocks - 1) / target_blocks;
    if (zc < 8) zc = 8;
    if (zc > IGR_FLUX_ZC_MAX) zc = IGR_FLUX_ZC_MAX;
    // on large grids twice the chunk, when at least 16 rounds of 256
    // blocks remain (fewer priming re-reads; 1024^3 FP64: 41.8 against
    // 42.4 ms per launch, while at 512^3 the 9 rounds it leaves lose 10 %)
    if (tiles * ((g.n[2] + 2 * IGR_FLUX_ZC_MAX - 1) / (2 * IGR_FLUX_ZC_MAX)) >= 16 * 256)
        zc = 2 * IGR_FLUX_ZC_MAX;
    if (zc > g.n[2]) zc = g.n[2];
    L.zc = int(zc);
    L.chunks = (g.n[2] + L.zc - 1) / L.zc;
    return L;
}

// The flux launch of storage form F (its shape follows the arithmetic type).
template <class F, int MODE, bool HASD = false>
int flux_impl(igr_ctx* c, const typename F::TB* U, const typename F::TD* D, const typename F::TS* sig,
              const typename F::TB* Un, FluxOut<F, MODE>* out, const double* dtp, double dt_fixed, hipStream_t s,
              double* speed = nullptr, typename F::TS* sig_out = nullptr) {
    using Sh = FluxShapeOf<F>;
    constexpr int TY = Sh::TY;
    const FluxLaunch L = flux_launch(c->g, TY, Sh::BLOCKS);
    if (L.blocks() > 0x7fffffffLL) return fail(IGR_EINVAL, "grid too large for the flux launch");
    return launch(c, K_FLUX, s, [&] {
        if (c->order == 3)
            k_flux_tiled<F, MODE, TY, 3, HASD><<<dim3(unsigned(L.blocks())), dim3(FLUX_TX, TY + 1), 0, s>>>(
                U, D, sig, Un, out, dtp, dt_fixed, c->g, c->d_flag, L.tiles_x, L.tiles_y, L.zc, speed, sig_out);
        else
            k_flux_tiled<F, MODE, TY, 5, HASD><<<dim3(unsigned(L.blocks())), dim3(FLUX_TX, TY + 1), 0, s>>>(
                U, D, sig, Un, out, dtp, dt_fixed, c->g, c->d_flag, L.tiles_x, L.tiles_y, L.zc, speed, sig_out);
    });
}

// blocks of one flux launch of form F (the length of the fused CFL maxima)
template <class F>
long long flux_blocks(const igr_ctx* c) {
    return flux_launch(c->g, FluxShapeOf<F>::TY, FluxShapeOf<F>::BLOCKS).blocks();
}

// Viscous terms added to `out` (the right-hand side, or the stage the
// flux kernel just wrote) from the stage input U: the stress, its ghosts,
// then the tiled viscous flux divergence.  Every form.  Tile
// heights (blocks of TY + 1 waves): FP64 7 (220-231 VGPRs at 2 waves per
// SIMD, no spill; 1024^3: 49.5-50.3 ms per launch, against 72 ms with the
// face stencils loaded whole and 108 ms without face sharing), FP32 11 (3
// waves per SIMD; 22.7 ms, TY = 8 about 4 ms more).  The stress kernel: 64 x 16 tiles
// (1024^3 FP64 16.2 ms, FP32 12.5 ms; TY = 8 19.8 / 13.9 ms; a column
// march without LDS 26.3 / 15.8 ms).
#ifndef IGR_VISC_TY_F64
#define IGR_VISC_TY_F64 7
#endif
#ifndef IGR_VISC_TY_F32
#define IGR_VISC_TY_F32 11
#endif
#ifndef IGR_VISC_MINW_F64
#define IGR_VISC_MINW_F64 2
#endif
#ifndef IGR_VISC_MINW_F32
#define IGR_VISC_MINW_F32 3
#endif
#ifndef IGR_STRESS_TY
#define IGR_STRESS_TY 16
#endif
#ifndef IGR_STRESS_BLOCKS
#define IGR_STRESS_BLOCKS 4096
#endif
#ifndef IGR_VISC_BLOCKS
#define IGR_VISC_BLOCKS 2048
#endif
// tile height of the viscous flux divergence of arithmetic type C
template <class C>
constexpr int visc_ty() {
    return sizeof(C) == 8 ? IGR_VISC_TY_F64 : IGR_VISC_TY_F32;
}
// blocks of one viscous flux-divergence launch of form F (the length of the
// CFL maxima its last stage leaves)
template <class F>
long long visc_blocks(const igr_ctx* c) {
    return flux_launch(c->g, visc_ty<typename F::C>(), IGR_VISC_BLOCKS).blocks();
}

// speed (last stage, nullable): the kernel also leaves the per-block CFL
// maxima of the new state there (visc_blocks values).
template <class F, int MODE, bool HASD = false>
int viscous_impl(igr_ctx* c, const typename F::TB* U, const typename F::TD* D, FluxOut<F, MODE>* out,
                 const double* dtp, double dt_fixed, hipStream_t s, double* speed = nullptr,
                 bool tau_ready = false) {
    {
        using C = typename F::C;
        constexpr int TY = visc_ty<C>();
        constexpr int MW = sizeof(C) == 8 ? IGR_VISC_MINW_F64 : IGR_VISC_MINW_F32;
        C* T6 = static_cast<C*>(c->d_G);
        const Geom& g = c->g;
        const FluxLaunch L = flux_launch(g, TY, IGR_VISC_BLOCKS);
        if (L.blocks() > 0x7fffffffLL) return fail(IGR_EINVAL, "grid too large for the viscous launch");
        const FluxLaunch LS = flux_launch(g, IGR_STRESS_TY, IGR_STRESS_BLOCKS);
        if (LS.blocks() > 0x7fffffffLL) return fail(IGR_EINVAL, "grid too large for the stress launch");
        // the stage's first Sigma pass may have stored the stress already
        if (!tau_ready)
            IGR_TRY(launch(c, K_STRESS, s, [&] {
                k_stress<F, IGR_STRESS_TY, HASD>
                    <<<dim3(unsigned(LS.blocks())), dim3(STRESS_TX, IGR_STRESS_TY), 0, s>>>(
                        U, D, T6, g, c->mu, c->zeta, LS.tiles_x, LS.tiles_y, LS.zc);
            }));
        for (int q = 0; q < 6; ++q) IGR_TRY(fill_sigma_ghosts(c, T6 + (size_t)q * g.fs, s));
        return launch(c, K_VISCOUS, s, [&] {
            const dim3 grid(unsigned(L.blocks())), block(VISC_TX, TY + 1);
            if (c->order == 3)
                k_viscous_tiled<F, MODE, TY, 3, MW, HASD><<<grid, block, 0, s>>>(
                    U, D, T6, out, dtp, dt_fixed, g, L.tiles_x, L.tiles_y, L.zc, speed, c->d_flag);
            else
                k_viscous_tiled<F, MODE, TY, 5, MW, HASD><<<grid, block, 0, s>>>(
                    U, D, T6, out, dtp, dt_fixed, g, L.tiles_x, L.tiles_y, L.zc, speed, c->d_flag);
        });
    }
}

template <class T>
int speed_dt_impl(igr_ctx* c, const T* U, double cfl, hipStream_t s) {
    IGR_TRY(launch(c, K_DT, s, [&] {
        k_speed_partial<T><<<RED_BLOCKS, RED_THREADS, 0, s>>>(U, c->g, c->d_partial, c->d_flag);
        k_dt_final<<<1, RED_THREADS, 0, s>>>(c->d_partial, RED_BLOCKS, cfl, c->d_scalars);
    }));
    return IGR_OK;
}

int read_flag(igr_ctx* c, hipStream_t s) {
    int flag = 0;
    IGR_HIP(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    IGR_HIP(hipStreamSynchronize(s));
    if (flag) {
        IGR_HIP(hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
        IGR_HIP(hipStreamSynchronize(s));
        return fail(IGR_ENONFINITE, "a kernel saw rho <= 0, p <= 0 or a non-finite value");
    }
    return IGR_OK;
}

template <class F>
int rhs_impl(igr_ctx* c, typename F::TB* U, typename F::TS* sig, typename F::TB* rhs, hipStream_t s) {
    IGR_TRY(fill_state_ghosts(c, U, s));
    IGR_TRY(sigma_solve_impl<F>(c, U, sig, c->nsweeps, s));
    IGR_TRY((flux_impl<F, MODE_RHS>(c, U, nullptr, sig, nullptr, rhs, nullptr, 0.0, s)));
    if (c->viscous) IGR_TRY((viscous_impl<F, MODE_RHS>(c, U, nullptr, rhs, nullptr, 0.0, s)));
    return IGR_OK;
}

// The three RK stages of one step from the state U (sigma: the previous
// stage's Sigma, in and out) with the time step at *dtp (device) or
// dt_fixed; with cfl_dt the time step is the CFL step of U, formed in stage
// 1 (dtp is then ignored).  With `speed` the last stage also leaves the
// per-block CFL maxima of the new state there (one value per flux block).
// The new state goes to Unew: the plain forms write it in place (Unew ==
// U); the split form writes it to the other FP32 state, because its last
// stage still reads U^n around every cell it writes.
// Sigma ping-pongs between the caller's buffer `sig` and the scratch copy;
// the step starts from sig_start (null: sig).  Without sig_end the solved
// Sigma ends in sig (the last flux stage copies it there when the solve
// ended in scratch); with sig_end it stays where the solve left it and
// *sig_end names that buffer (a later step starts from it).
template <class F>
int step_stages(igr_ctx* c, typename F::TB* U, typename F::TB* Unew, typename F::TS* sig, const double* dtp,
                double dt_fixed, hipStream_t s, double* speed, bool cfl_dt = false, double cfl = 0.0,
                typename F::TS* sig_start = nullptr, typename F::TS** sig_end = nullptr) {
    using TD = typename F::TD;
    using TS = typename F::TS;
    TD* Ua = static_cast<TD*>(c->d_Ua);
    TD* Ub = static_cast<TD*>(c->d_Ub);
    TS* cur = sig_start ? sig_start : sig;
    TS* oth = cur == sig ? static_cast<TS*>(c->d_sig2) : sig;
    // with viscous terms the stage's first two-level Sigma pass also stores
    // the stress of the stage input (tau: whether it did)
    using C = typename F::C;
    C* T6 = c->viscous ? static_cast<C*>(c->d_G) : nullptr;
    bool tau = false;
    auto solve = [&](auto hasd, const typename F::TB* Us, const TD* Ds, double* spd = nullptr,
                     int* nspd = nullptr) -> int {
        TS* res = nullptr;
        IGR_TRY((sigma_solve_buf<F, decltype(hasd)::value>(c, Us, Ds, cur, oth, c->nsweeps, &res, s, spd, nspd, T6,
                                                           &tau)));
        if (res != cur) {
            oth = cur;
            cur = res;
        }
        return IGR_OK;
    };
    using NoD = std::false_type;
    // the later stages read U^n + difference in the split form
    using LaterD = std::integral_constant<bool, F::SPLIT>;
    // stage 1: U1 = Un + dt L(Un)
    IGR_TRY(fill_state_ghosts(c, U, s));
    if (cfl_dt) {
        // dt from Un: the first sweep of this solve forms the CFL maxima
        // when it can (FP64, solve starting with a single sweep), else the
        // standalone reduction runs; either way before the flux needs dt
        int nspd = 0;
        IGR_TRY(solve(NoD{}, U, nullptr, c->d_speed, &nspd));
        if (nspd > 0)
            IGR_TRY(launch(c, K_DT, s, [&] {
                k_dt_final<<<1, RED_THREADS, 0, s>>>(c->d_speed, nspd, cfl, c->d_scalars);
            }));
        else
            IGR_TRY(speed_dt_impl(c, (const typename F::TB*)U, cfl, s));
        dtp = c->d_scalars;
    } else {
        IGR_TRY(solve(NoD{}, U, nullptr));
    }
    IGR_TRY((flux_impl<F, MODE_STAGE1>(c, U, nullptr, cur, nullptr, Ua, dtp, dt_fixed, s)));
    if (c->viscous) IGR_TRY((viscous_impl<F, MODE_STAGE1>(c, U, nullptr, Ua, dtp, dt_fixed, s, nullptr, tau)));
    if constexpr (F::SPLIT) {
        // stage 2: U2 - Un = 1/4 ((U1 - Un) + dt L(U1)), U1 = Un + Ua
        IGR_TRY(fill_state_ghosts(c, Ua, s, true));
        IGR_TRY(solve(LaterD{}, U, Ua));
        IGR_TRY((flux_impl<F, MODE_STAGE2, true>(c, U, Ua, cur, nullptr, Ub, dtp, dt_fixed, s)));
        if (c->viscous) IGR_TRY((viscous_impl<F, MODE_STAGE2, true>(c, U, Ua, Ub, dtp, dt_fixed, s, nullptr, tau)));
        // stage 3: Un+1 = Un + 2/3 ((U2 - Un) + dt L(U2)), U2 = Un + Ub
        IGR_TRY(fill_state_ghosts(c, Ub, s, true));
        IGR_TRY(solve(LaterD{}, U, Ub));
        IGR_TRY((flux_impl<F, MODE_STAGE3, true>(c, U, Ub, cur, nullptr, Unew, dtp, dt_fixed, s,
                                                 c->viscous ? nullptr : speed, !sig_end && cur != sig ? sig : nullptr)));
        if (c->viscous) IGR_TRY((viscous_impl<F, MODE_STAGE3, true>(c, U, Ub, Unew, dtp, dt_fixed, s, speed, tau)));
    } else {
        // stage 2: U2 = 3/4 Un + 1/4 (U1 + dt L(U1))
        IGR_TRY(fill_state_ghosts(c, Ua, s));
        IGR_TRY(solve(NoD{}, Ua, nullptr));
        IGR_TRY((flux_impl<F, MODE_STAGE2>(c, Ua, nullptr, cur, U, Ub, dtp, dt_fixed, s)));
        if (c->viscous) IGR_TRY((viscous_impl<F, MODE_STAGE2>(c, Ua, nullptr, Ub, dtp, dt_fixed, s, nullptr, tau)));
        // stage 3: Un+1 = 1/3 Un + 2/3 (U2 + dt L(U2)), in place over Un; if the
        // solve ended in the scratch copy the kernel also writes Sigma's interior
        // into the caller's buffer (its ghosts are scratch)
        IGR_TRY(fill_state_ghosts(c, Ub, s));
        IGR_TRY(solve(NoD{}, Ub, nullptr));
        // with viscous terms their kernel, which completes the new state,
        // forms the CFL maxima instead of the flux kernel
        IGR_TRY((flux_impl<F, MODE_STAGE3>(c, Ub, nullptr, cur, U, Unew, dtp, dt_fixed, s,
                                           c->viscous ? nullptr : speed, !sig_end && cur != sig ? sig : nullptr)));
        if (c->viscous) IGR_TRY((viscous_impl<F, MODE_STAGE3>(c, Ub, nullptr, Unew, dtp, dt_fixed, s, speed, tau)));
    }
    if (sig_end) *sig_end = cur;
    return IGR_OK;
}

// The state a step writes: in place, or the split form's other FP32 state.
template <class F>
typename F::TB* next_state(igr_ctx* c, typename F::TB* U, typename F::TB* Ucaller) {
    if constexpr (F::SPLIT)
        return U == Ucaller ? static_cast<typename F::TB*>(c->d_Unb) : Ucaller;
    else
        return U;
}

// Copies a split-form result from the other FP32 state into the caller's U.
template <class F>
int settle_state(igr_ctx* c, typename F::TB* U, typename F::TB* Ucaller, hipStream_t s) {
    if (U != Ucaller)
        IGR_HIP(hipMemcpyAsync(Ucaller, U, 5 * field_bytes(c, sizeof(typename F::TB)), hipMemcpyDeviceToDevice, s));
    return IGR_OK;
}

template <class F>
int step_impl(igr_ctx* c, typename F::TB* U, typename F::TS* sig, double cfl, double dt_fixed, hipStream_t s) {
    typename F::TB* Unew = next_state<F>(c, U, U);
    if (!(dt_fixed > 0.0))
        IGR_TRY(step_stages<F>(c, U, Unew, sig, nullptr, dt_fixed, s, nullptr, true, cfl));
    else
        IGR_TRY(step_stages<F>(c, U, Unew, sig, nullptr, dt_fixed, s, nullptr));
    return settle_state<F>(c, Unew, U, s);
}

// nsteps steps.  With a CFL time step the first step's maximum comes from
// the standalone reduction and every later one from the maxima that the
// previous step's last stage left in d_speed (the flux kernel's, or with
// viscous terms the viscous kernel's, which completes the new state).  The
// split form alternates between the caller's U and its other FP32 state
// and copies the last state into U if it ends in the other one.
template <class F>
int advance_impl(igr_ctx* c, typename F::TB* Ucaller, typename F::TS* sig, int nsteps, double cfl, double dt_fixed,
                 hipStream_t s) {
    using TB = typename F::TB;
    const bool use_cfl = !(dt_fixed > 0.0);
    const int nblk = int(c->viscous ? visc_blocks<F>(c) : flux_blocks<F>(c));
    TB* U = Ucaller;
    // Sigma stays where a step's solve left it until the last step, which
    // ends it in the caller's buffer
    typename F::TS* scur = sig;
    for (int n = 0; n < nsteps; ++n) {
        TB* Unew = next_state<F>(c, U, Ucaller);
        const bool last = n + 1 == nsteps;
        const double* dtp = nullptr;
        if (use_cfl) {
            if (n == 0) {
                IGR_TRY(speed_dt_impl(c, (const TB*)U, cfl, s));
            } else {
                IGR_TRY(launch(c, K_DT, s, [&] {
                    k_dt_final<<<1, RED_THREADS, 0, s>>>(c->d_speed, nblk, cfl, c->d_scalars);
                }));
            }
            dtp = c->d_scalars;
        }
        IGR_TRY(step_stages<F>(c, U, Unew, sig, dtp, dt_fixed, s, use_cfl && !last ? c->d_speed : nullptr, false, 0.0,
                               scur, last ? nullptr : &scur));
        U = Unew;
    }
    return settle_state<F>(c, U, Ucaller, s);
}

template <class T>
int sums_impl(igr_ctx* c, const T* U, double out[5], hipStream_t s) {
    IGR_TRY(launch(c, K_SUMS, s, [&] {
        k_sums_partial<T><<<RED_BLOCKS, RED_THREADS, 0, s>>>(U, c->g, c->d_partial);
        k_sum_final<5><<<1, RED_THREADS, 0, s>>>(c->d_partial, RED_BLOCKS, c->dx * c->dy * c->dz, c->d_scalars + 1);
    }));
    IGR_HIP(hipMemcpyAsync(out, c->d_scalars + 1, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
    IGR_HIP(hipStreamSynchronize(s));
    return IGR_OK;
}

template <class F>
int resid_impl(igr_ctx* c, const typename F::TB* U, const typename F::TS* sig, double* out, hipStream_t s) {
    using C = typename F::C;
    const C* b = static_cast<const C*>(c->d_b);
    IGR_TRY(launch(c, K_RESID, s, [&] {
        k_resid_partial<typename F::TS, typename F::TB, C>
            <<<RED_BLOCKS, RED_THREADS, 0, s>>>(sig, b, U, c->g, c->d_partial);
        k_sum_final<1><<<1, RED_THREADS, 0, s>>>(c->d_partial, RED_BLOCKS, 1.0, c->d_scalars + 6);
    }));
    double r2 = 0.0;
    IGR_HIP(hipMemcpyAsync(&r2, c->d_scalars + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    IGR_HIP(hipStreamSynchronize(s));
    *out = std::sqrt(r2);
    return IGR_OK;
}

// Per-column owner/chi of the x-min inflow discs (host, FP64).
int upload_patches(igr_ctx* c) {
    const int ny = c->ny, nz = c->nz;
    std::vector<int> owner((size_t)ny * nz, -1);
    std::vector<double> chi((size_t)ny * nz, 0.0);
    for (int k = 0; k < nz; ++k) {
        for (int j = 0; j < ny; ++j) {
            const double y = (j + 0.5) * c->dy, z = (k + 0.5) * c->dz;
            double best = INFINITY;
            int q = -1;
            for (size_t p = 0; p < c->patches.size(); ++p) {
                const double ey = y - c->patches[p].yc, ez = z - c->patches[p].zc;
                const double d2 = ey * ey + ez * ez;
                if (d2 < best) {
                    best = d2;
                    q = int(p);
                }
            }
            owner[(size_t)k * ny + j] = q;
            if (q >= 0) {
                const igr_patch& pa = c->patches[q];
                chi[(size_t)k * ny + j] = pa.width > 0 ? 0.5 * (1.0 - std::tanh((std::sqrt(best) - pa.r) / pa.width))
                                                       : (best <= pa.r * pa.r ? 1.0 : 0.0);
            }
        }
    }
    c->h_owner = owner;
    IGR_HIP(hipMemcpy(c->d_owner, owner.data(), owner.size() * sizeof(int), hipMemcpyHostToDevice));
    IGR_HIP(hipMemcpy(c->d_chi, chi.data(), chi.size() * sizeof(double), hipMemcpyHostToDevice));
    return IGR_OK;
}

int upload_jets(igr_ctx* c, hipStream_t s, bool sync) {
    if (c->patches.empty()) return IGR_OK;
    std::vector<double> jet(c->patches.size() * 5);
    const double gm = c->g.gamma;
    for (size_t p = 0; p < c->patches.size(); ++p) {
        const igr_patch& pa = c->patches[p];
        jet[p * 5 + 0] = pa.rho;
        jet[p * 5 + 1] = pa.rho * pa.ux;
        jet[p * 5 + 2] = pa.rho * pa.uy;
        jet[p * 5 + 3] = pa.rho * pa.uz;
        jet[p * 5 + 4] = pa.p / (gm - 1.0) + 0.5 * pa.rho * (pa.ux * pa.ux + pa.uy * pa.uy + pa.uz * pa.uz);
    }
    IGR_HIP(hipMemcpyAsync(c->d_jet, jet.data(), jet.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if (sync) IGR_HIP(hipStreamSynchronize(s));
    return IGR_OK;
}

void release(igr_ctx* c) {
    if (!c) return;
    void* ptrs[] = {c->d_owner, c->d_chi,     c->d_jet,      c->d_Ua,   c->d_Ub,    c->d_sig2, c->d_b,
                    c->d_ir,    c->d_partial, c->d_scalars,  c->d_flag, c->d_speed, c->d_Unb,  c->d_jet0,
                    c->d_G};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (double* p : c->adj)
        if (p) (void)hipFree(p);
    for (auto& r : c->records) {
        c->event_pool.push_back(r.start);
        c->event_pool.push_back(r.stop);
    }
    for (hipEvent_t e : c->event_pool)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

#define DISPATCH(ctx, FN, ...)                                                                        \
    ((ctx)->precision == IGR_F64          ? FN<Plain<double>>(__VA_ARGS__)                            \
     : (ctx)->precision == IGR_F32        ? FN<Plain<float>>(__VA_ARGS__)                             \
     : (ctx)->precision == IGR_F16_F32    ? FN<Plain<f16>>(__VA_ARGS__)                               \
     : (ctx)->precision == IGR_F32_BF16D  ? FN<Split>(__VA_ARGS__)                                    \
                                          : FN<Plain<bf16>>(__VA_ARGS__))

template <class F>
int rhs_t(igr_ctx* c, void* U, void* sig, void* rhs, hipStream_t s) {
    return rhs_impl<F>(c, static_cast<typename F::TB*>(U), static_cast<typename F::TS*>(sig),
                       static_cast<typename F::TB*>(rhs), s);
}
template <class F>
int step_t(igr_ctx* c, void* U, void* sig, double cfl, double dt_fixed, hipStream_t s) {
    return step_impl<F>(c, static_cast<typename F::TB*>(U), static_cast<typename F::TS*>(sig), cfl, dt_fixed, s);
}
template <class F>
int advance_t(igr_ctx* c, void* U, void* sig, int nsteps, double cfl, double dt_fixed, hipStream_t s) {
    return advance_impl<F>(c, static_cast<typename F::TB*>(U), static_cast<typename F::TS*>(sig), nsteps, cfl,
                           dt_fixed, s);
}
template <class F>
int sigma_t(igr_ctx* c, void* U, void* sig, int nsweeps, double* resid, hipStream_t s) {
    using TB = typename F::TB;
    using TS = typename F::TS;
    IGR_TRY(fill_state_ghosts(c, static_cast<TB*>(U), s));
    IGR_TRY(sigma_solve_impl<F>(c, static_cast<TB*>(U), static_cast<TS*>(sig), nsweeps, s));
    if (resid) {
        IGR_TRY(source_impl(c, static_cast<const TB*>(U), s));
        IGR_TRY(resid_impl<F>(c, static_cast<const TB*>(U), static_cast<const TS*>(sig), resid, s));
    }
    return IGR_OK;
}
template <class F>
int dt_t(igr_ctx* c, const void* U, double cfl, hipStream_t s) {
    return speed_dt_impl(c, static_cast<const typename F::TB*>(U), cfl, s);
}
template <class F>
int sums_t(igr_ctx* c, const void* U, double* out, hipStream_t s) {
    return sums_impl(c, static_cast<const typename F::TB*>(U), out, s);
}

// ---------------------------------------------------------------------------
// Adjoint (FP64)
// ---------------------------------------------------------------------------

// Adjoint scratch: fields of the padded size (index -> role)
enum AdjBuf {
    A_U1, A_U2 = A_U1 + 5, A_SIG1 = A_U2 + 5, A_SIG2, A_SPAD, A_UBPAD, A_SBPAD = A_UBPAD + 5, A_FA,
    A_NB = A_FA + 12, A_DB, A_BB, A_IR, A_IRB, A_LB, A_UST = A_LB + 5, A_SBA = A_UST + 5, A_SBB, A_UBN,
    A_UB1 = A_UBN + 5, A_UB2 = A_UB1 + 5, A_UBIN = A_UB2 + 5, A_SBIN = A_UBIN + 5, A_ITER
};
// Viscous adjoint scratch (a second block, viscous contexts only): face
// cotangents (14), tau-bar with ghosts (6), folded tau-bar (6), G-bar (9),
// a field of zeros
enum ViscAdjBuf { V_FV, V_TB = V_FV + 14, V_TF = V_TB + 6, V_GB = V_TF + 6, V_ZERO = V_GB + 9, V_COUNT };

int adjoint_buffers(igr_ctx* c) {
    const int S = c->nsweeps;
    if (c->adj_sweeps == S) return IGR_OK;
    for (double* p : c->adj)
        if (p) (void)hipFree(p);
    c->adj.clear();
    const int nfield = A_ITER + S + 1;
    double* base = nullptr;
    hipError_t e = hipMalloc((void**)&base, (size_t)nfield * field_bytes(c, sizeof(double)) +
                                               (size_t)c->ny * c->nz * 5 * sizeof(double));
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? IGR_ENOMEM : IGR_EHIP,
                                     std::string("adjoint scratch: ") + hipGetErrorString(e));
    c->adj.push_back(base);
    IGR_HIP(hipMemset(base, 0, (size_t)nfield * field_bytes(c, sizeof(double))));
    if (c->viscous) {
        double* vb = nullptr;
        e = hipMalloc((void**)&vb, (size_t)V_COUNT * field_bytes(c, sizeof(double)));
        if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? IGR_ENOMEM : IGR_EHIP,
                                         std::string("viscous adjoint scratch: ") + hipGetErrorString(e));
        c->adj.push_back(vb);
        IGR_HIP(hipMemset(vb, 0, (size_t)V_COUNT * field_bytes(c, sizeof(double))));
    }
    c->adj_sweeps = S;
    return IGR_OK;
}

double* abuf(igr_ctx* c, int idx) { return c->adj[0] + (size_t)idx * c->g.fs; }

double* vbuf(igr_ctx* c, int idx) { return c->adj[1] + (size_t)idx * c->g.fs; }
double* ajetcol(igr_ctx* c) { return c->adj[0] + (size_t)(A_ITER + c->nsweeps + 1) * c->g.fs; }

dim3 padded_grid(const Geom& g) { return dim3((g.n[0] + 2 * G + 63) / 64, (g.n[1] + 2 * G + 3) / 4, g.n[2] + 2 * G); }

int axpby(igr_ctx* c, double a, const double* x, double b, double* y, int nf, hipStream_t s) {
    return launch(c, K_ADJOINT, s, [&] { k_axpby<<<cell_grid(c->g), cell_block(), 0, s>>>(a, x, b, y, nf, c->g); });
}

int dcopy(igr_ctx* c, double* dst, const double* src, int nf, hipStream_t s) {
    IGR_HIP(hipMemcpyAsync(dst, src, (size_t)nf * field_bytes(c, sizeof(double)), hipMemcpyDeviceToDevice, s));
    return IGR_OK;
}

int dzero(igr_ctx* c, double* p, int nf, hipStream_t s) {
    IGR_HIP(hipMemsetAsync(p, 0, (size_t)nf * field_bytes(c, sizeof(double)), s));
    return IGR_OK;
}

// Viscous part of a right-hand side's adjoint: adds into Ubpad (padded
// state cotangent) what L_v(U) contributes for the cotangent Lb.  U's
// ghosts are filled; the stress of U is formed again into d_G.
int viscous_adjoint(igr_ctx* c, const double* U, const double* Lb, double* Ubpad, hipStream_t s) {
    using F = Plain<double>;
    const Geom& g = c->g;
    double* T6 = static_cast<double*>(c->d_G);
    double* FV = vbuf(c, V_FV);
    double* Tb = vbuf(c, V_TB);
    double* Tf = vbuf(c, V_TF);
    double* Gb = vbuf(c, V_GB);
    const double* Z = vbuf(c, V_ZERO);
    const FluxLaunch LS = flux_launch(g, IGR_STRESS_TY, IGR_STRESS_BLOCKS);
    IGR_TRY(launch(c, K_ADJOINT, s, [&] {
        k_stress<F, IGR_STRESS_TY, false><<<dim3(unsigned(LS.blocks())), dim3(STRESS_TX, IGR_STRESS_TY), 0, s>>>(
            U, nullptr, T6, g, c->mu, c->zeta, LS.tiles_x, LS.tiles_y, LS.zc);
    }));
    for (int q = 0; q < 6; ++q) IGR_TRY(fill_sigma_ghosts(c, T6 + (size_t)q * g.fs, s));
    IGR_TRY(dzero(c, Tb, 6, s));
    for (int d = 0; d < 3; ++d) {
        const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
        const long long lines = (long long)g.n[a] * g.n[b];
        const int bf = int((lines * (g.n[d] + 1) + 255) / 256);
        const int bg = int((lines * (g.n[d] + 2 * G) + 255) / 256);
        auto faces = [&](auto dd, auto order) {
            constexpr int DD = decltype(dd)::value, OR = decltype(order)::value;
            k_adj_visc_face<DD, OR><<<bf, 256, 0, s>>>(U, T6, Lb, FV, g);
            k_adj_visc_gather<DD, OR><<<bg, 256, 0, s>>>(FV, Ubpad, Tb, g);
        };
        IGR_TRY(launch(c, K_ADJOINT, s, [&] {
            using O3 = std::integral_constant<int, 3>;
            using O5 = std::integral_constant<int, 5>;
            if (d == 0) {
                if (c->order == 3) faces(std::integral_constant<int, 0>{}, O3{});
                else faces(std::integral_constant<int, 0>{}, O5{});
            } else if (d == 1) {
                if (c->order == 3) faces(std::integral_constant<int, 1>{}, O3{});
                else faces(std::integral_constant<int, 1>{}, O5{});
            } else {
                if (c->order == 3) faces(std::integral_constant<int, 2>{}, O3{});
                else faces(std::integral_constant<int, 2>{}, O5{});
            }
        }));
    }
    // tau's ghost copies folded back (the rule is Sigma's), then tau(G) and
    // the central differences of u
    IGR_TRY(launch(c, K_ADJOINT, s, [&] {
        for (int q = 0; q < 6; ++q)
            k_adj_sigma_bc<<<cell_grid(g), cell_block(), 0, s>>>(Tb + (size_t)q * g.fs, Z, Tf + (size_t)q * g.fs, g);
    }));
    IGR_TRY(dzero(c, Gb, 9, s));
    const dim3 ugrid(unsigned((g.n[0] + 2 + 63) / 64), unsigned((g.n[1] + 2 + 3) / 4), unsigned(g.n[2] + 2));
    IGR_TRY(launch(c, K_ADJOINT, s, [&] {
        k_adj_stress_g<<<cell_grid(g), cell_block(), 0, s>>>(Tf, Gb, g, c->mu, c->zeta);
        k_adj_stress_u<<<ugrid, cell_block(), 0, s>>>(U, Gb, Ubpad, g);
    }));
    return IGR_OK;
}

// Adjoint of one right-hand side (L, Sigma_new) = RHS(U, Sigma_p):
// given L-bar (Lb, 5 fields) and Sigma_new-bar (Sbn), write U-bar (Ub_out,
// interior, 5 fields) and Sigma_p-bar (Sbp_out, interior); add the x-min
// jet cotangents (conserved, per patch) to jbar.
int stage_adjoint(igr_ctx* c, double* U, const double* Sp, const double* Lb, const double* Sbn, double* Ub_out,
                  double* Sbp_out, std::vector<double>& jbar, hipStream_t s) {
    const Geom& g = c->g;
    const int S = c->nsweeps;
    double* ir = abuf(c, A_IR);
    double* Spad = abuf(c, A_SPAD);
    double* Ubpad = abuf(c, A_UBPAD);
    double* Sbpad = abuf(c, A_SBPAD);
    double* FA = abuf(c, A_FA);
    double* Nb = abuf(c, A_NB);
    double* Db = abuf(c, A_DB);
    double* bb = abuf(c, A_BB);
    double* irb = abuf(c, A_IRB);
    double* sbA = abuf(c, A_SBA);
    double* sbB = abuf(c, A_SBB);
    auto iter = [&](int k) { return abuf(c, A_ITER + k); };
    // forward recompute: ghosts, 1/rho, the S sweep iterates
    IGR_TRY(fill_state_ghosts(c, U, s));
    IGR_TRY(launch(c, K_ADJOINT, s, [&] { k_inv_rho<<<padded_grid(g), cell_block(), 0, s>>>(U, ir, g); }));
    IGR_TRY(dcopy(c, iter(0), Sp, 1, s));
    IGR_TRY(source_impl(c, (const double*)U, s));
    for (int k = 1; k <= S; ++k)
        IGR_TRY(launch(c, K_SWEEP, s, [&] {
            k_jacobi<double, double><<<cell_grid(g), cell_block(), 0, s>>>(iter(k - 1), iter(k),
                                                                           (const double*)c->d_b, U, g);
        }));
    IGR_TRY(dcopy(c, Spad, iter(S), 1, s));
    IGR_TRY(fill_sigma_ghosts(c, Spad, s));
    // flux: per direction, face cotangents then the transposed stencil
    IGR_TRY(dzero(c, Ubpad, 5, s));
    IGR_TRY(dzero(c, Sbpad, 1, s));
    for (int d = 0; d < 3; ++d) {
        const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
        const long long lines = (long long)g.n[a] * g.n[b];
        const int bf = int((lines * (g.n[d] + 1) + 255) / 256);
        const int bg = int((lines * (g.n[d] + 2 * G) + 255) / 256);
        auto faces = [&](auto dd, auto order) {
            constexpr int DD = decltype(dd)::value, OR = decltype(order)::value;
            k_adj_face<DD, OR><<<bf, 256, 0, s>>>(U, Spad, Lb, FA, g);
            k_adj_recon_gather<DD, OR><<<bg, 256, 0, s>>>(FA, Ubpad, Sbpad, g);
        };
        IGR_TRY(launch(c, K_ADJOINT, s, [&] {
            using O3 = std::integral_constant<int, 3>;
            using O5 = std::integral_constant<int, 5>;
            if (d == 0) {
                if (c->order == 3) faces(std::integral_constant<int, 0>{}, O3{});
                else faces(std::integral_constant<int, 0>{}, O5{});
            } else if (d == 1) {
                if (c->order == 3) faces(std::integral_constant<int, 1>{}, O3{});
                else faces(std::integral_constant<int, 1>{}, O5{});
            } else {
                if (c->order == 3) faces(std::integral_constant<int, 2>{}, O3{});
                else faces(std::integral_constant<int, 2>{}, O5{});
            }
        }));
    }
    if (c->viscous) IGR_TRY(viscous_adjoint(c, U, Lb, Ubpad, s));
    // Sigma ghosts transposed: sbA = Sigma^S-bar
    IGR_TRY(launch(c, K_ADJOINT, s, [&] { k_adj_sigma_bc<<<cell_grid(g), cell_block(), 0, s>>>(Sbpad, Sbn, sbA, g); }));
    // Jacobi levels in reverse
    IGR_TRY(dzero(c, bb, 1, s));
    IGR_TRY(dzero(c, irb, 1, s));
    for (int k = S; k >= 1; --k) {
        IGR_TRY(launch(c, K_ADJOINT, s, [&] {
            k_adj_jac1<<<cell_grid(g), cell_block(), 0, s>>>(sbA, iter(k), ir, Nb, Db, bb, g);
            k_adj_jac2<<<padded_grid(g), cell_block(), 0, s>>>(Nb, Db, iter(k - 1), ir, sbB, irb, g);
        }));
        double* t = sbA;
        sbA = sbB;
        sbB = t;
    }
    IGR_TRY(dcopy(c, Sbp_out, sbA, 1, s));
    // source, 1/rho, ghosts of U
    IGR_TRY(launch(c, K_ADJOINT, s, [&] {
        k_adj_source<<<padded_grid(g), cell_block(), 0, s>>>(U, ir, bb, Ubpad, irb, g);
        k_adj_irho<<<padded_grid(g), cell_block(), 0, s>>>(ir, irb, Ubpad, g);
    }));
    const bool inflow = !c->patches.empty();
    double* jc = ajetcol(c);
    IGR_TRY(launch(c, K_ADJOINT, s, [&] {
        k_adj_bc_state<<<cell_grid(g), cell_block(), 0, s>>>(Ubpad, Ub_out, inflow ? c->d_owner : nullptr, c->d_chi,
                                                             inflow ? jc : nullptr, g);
    }));
    if (inflow) {
        const size_t cols = (size_t)c->ny * c->nz;
        std::vector<double> h(cols * 5);
        IGR_HIP(hipMemcpyAsync(h.data(), jc, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        IGR_HIP(hipStreamSynchronize(s));
        for (size_t col = 0; col < cols; ++col) {
            const int q = c->h_owner[col];
            if (q < 0) continue;
            for (int f = 0; f < 5; ++f) jbar[(size_t)q * 5 + f] += h[col * 5 + f];
        }
    }
    return IGR_OK;
}

// conserved jet cotangents -> primitive (rho, ux, uy, uz, p) cotangents
void jet_primitive_bar(const igr_ctx* c, const std::vector<double>& jbar, double* out) {
    const double g1 = c->g.gamma - 1.0;
    for (size_t q = 0; q < c->patches.size(); ++q) {
        const igr_patch& pa = c->patches[q];
        const double* J = &jbar[q * 5];
        const double u[3] = {pa.ux, pa.uy, pa.uz};
        const double ke = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        out[q * 5 + 0] = J[0] + J[1] * u[0] + J[2] * u[1] + J[3] * u[2] + J[4] * ke;
        for (int k = 0; k < 3; ++k) out[q * 5 + 1 + k] = J[1 + k] * pa.rho + J[4] * pa.rho * u[k];
        out[q * 5 + 4] = J[4] / g1;
    }
}


// ---------------------------------------------------------------------------
// Allocation-free CFL time step (igr_compute_dt_noalloc)
// ---------------------------------------------------------------------------

// Scratch of the allocation-free entry point: RED_BLOCKS FP64 partial maxima,
// the FP64 result and the non-finite flag.  Each device the library runs on
// holds its own copy until the process ends.  In host code this name is a
// host-side stand-in, never a device address: host code uses the address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocPartialOff = 0;
constexpr size_t kNoAllocResultOff = RED_BLOCKS * sizeof(double);
constexpr size_t kNoAllocFlagOff = kNoAllocResultOff + sizeof(double);
constexpr size_t kNoAllocBytes = 16384;
static_assert(kNoAllocFlagOff + sizeof(int) <= kNoAllocBytes, "scratch too small for the reduction");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// Conserved state of inflow disc q (stream-ordered update of the jet table).
__global__ void k_set_jet(double* jet, int q, double r, double mx, double my, double mz, double E) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        jet[q * 5 + 0] = r;
        jet[q * 5 + 1] = mx;
        jet[q * 5 + 2] = my;
        jet[q * 5 + 3] = mz;
        jet[q * 5 + 4] = E;
    }
}

__global__ void k_clear_flag(int* flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = 0;
}

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
unsigned char* g_noalloc_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int noalloc_scratch(unsigned char** out) {
    int dev = 0;
    IGR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(IGR_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        IGR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(IGR_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
        g_noalloc_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_noalloc_ptr[dev];
    return IGR_OK;
}

template <class T>
int dt_noalloc_t(const Geom& g, const void* U, double* partial, double* result, int* flag, double cfl,
                 hipStream_t s) {
    k_clear_flag<<<1, 64, 0, s>>>(flag);
    k_speed_partial<T><<<RED_BLOCKS, RED_THREADS, 0, s>>>(static_cast<const T*>(U), g, partial, flag);
    k_dt_final<<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, cfl, result);
    IGR_HIP(hipGetLastError());
    return IGR_OK;
}

}  // namespace

extern "C" {

const char* igr_last_error(void) { return g_last_error.c_str(); }

const char* igr_kernel_name(int32_t index) {
    if (index < 0 || index >= K_COUNT) return nullptr;
    return kKernelNames[index];
}

int igr_init(const igr_grid* grid, double gamma, double alpha, const igr_bc* bc, const igr_opts* opts,
             igr_ctx** out) {
    if (!grid || !bc || !opts || !out) return fail(IGR_EINVAL, "null argument");
    *out = nullptr;
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(IGR_EINVAL, "grid extents must be >= 1");
    if (!(grid->dx > 0) || !(grid->dy > 0) || !(grid->dz > 0)) return fail(IGR_EINVAL, "spacings must be > 0");
    if (!(gamma > 1.0)) return fail(IGR_EINVAL, "gamma must be > 1");
    if (!(alpha >= 0.0)) return fail(IGR_EINVAL, "alpha must be >= 0");
    for (int f = 0; f < 6; ++f)
        if (bc->face[f] != IGR_BC_PERIODIC && bc->face[f] != IGR_BC_EXTRAP) return fail(IGR_EINVAL, "unknown face kind");
    for (int d = 0; d < 3; ++d)
        if ((bc->face[2 * d] == IGR_BC_PERIODIC) != (bc->face[2 * d + 1] == IGR_BC_PERIODIC))
            return fail(IGR_EINVAL, "periodic faces must come in pairs");
    if (bc->npatch < 0 || (bc->npatch > 0 && !bc->patch)) return fail(IGR_EINVAL, "bad patch list");
    if (bc->npatch > 0 && bc->face[0] == IGR_BC_PERIODIC) return fail(IGR_EINVAL, "inflow discs need a non-periodic x axis");
    for (int p = 0; p < bc->npatch; ++p) {
        const igr_patch& pa = bc->patch[p];
        if (!(pa.r >= 0) || !(pa.width >= 0) || !(pa.rho > 0) || !(pa.p > 0))
            return fail(IGR_EINVAL, "inflow disc needs r >= 0, width >= 0, rho > 0, p > 0");
    }
    if (opts->precision != IGR_F64 && opts->precision != IGR_F32 && opts->precision != IGR_BF16_F32 &&
        opts->precision != IGR_F16_F32 && opts->precision != IGR_F32_BF16D)
        return fail(IGR_EINVAL, "unknown precision");
    if (opts->precision == IGR_F32_BF16D && opts->sigma_block > 2)
        return fail(IGR_EUNSUPPORTED, "IGR_F32_BF16D runs single or two-sweep Sigma passes (sigma_block 0..2)");
    if (!(opts->mu >= 0.0) || !(opts->zeta >= 0.0)) return fail(IGR_EINVAL, "viscosities must be >= 0");
    if (opts->order != 5 && opts->order != 3)
        return fail(IGR_EUNSUPPORTED, "reconstruction order must be 5 or 3");
    if (opts->nsweeps < 0) return fail(IGR_EINVAL, "nsweeps must be >= 0");
    if (opts->sigma_block < 0 || opts->sigma_block > 5) return fail(IGR_EINVAL, "sigma_block must be in 0..5");
    if (opts->smoother != IGR_SMOOTH_JACOBI && opts->smoother != IGR_SMOOTH_RBGS)
        return fail(IGR_EINVAL, "unknown smoother");
    if (opts->smoother == IGR_SMOOTH_RBGS) {
        const int ext[3] = {grid->nx, grid->ny, grid->nz};
        for (int d = 0; d < 3; ++d)
            if (bc->face[2 * d] == IGR_BC_PERIODIC && (ext[d] & 1))
                return fail(IGR_EUNSUPPORTED, "red-black Gauss-Seidel needs even extents on periodic axes");
    }

    igr_ctx* c = new (std::nothrow) igr_ctx();
    if (!c) return fail(IGR_ENOMEM, "host allocation failed");
    c->nx = grid->nx;
    c->ny = grid->ny;
    c->nz = grid->nz;
    c->dx = grid->dx;
    c->dy = grid->dy;
    c->dz = grid->dz;
    c->precision = opts->precision;
    c->nsweeps = opts->nsweeps;
    c->order = opts->order;
    c->smoother = opts->smoother;
    c->mu = opts->mu;
    c->zeta = opts->zeta;
    c->viscous = opts->mu > 0.0 || opts->zeta > 0.0;
    c->sigma_block = opts->sigma_block;   // 0: resolved below, once the field size is known
    for (int f = 0; f < 6; ++f) c->faces[f] = bc->face[f];
    c->patches.assign(bc->patch, bc->patch + bc->npatch);
    const long long px = grid->nx + 2 * G, py = grid->ny + 2 * G, pz = grid->nz + 2 * G;
    Geom& g = c->g;
    g.n[0] = grid->nx;
    g.n[1] = grid->ny;
    g.n[2] = grid->nz;
    // kernels address a plane with 32-bit byte offsets (8-byte elements)
    if (px * py > (1LL << 29) - 1) {
        delete c;
        return fail(IGR_EINVAL, "x-y plane too large");
    }
    g.st[0] = 1;
    g.st[1] = int(px);
    g.st[2] = int(px * py);
    g.fs = px * py * pz;
    g.ih[0] = 1.0 / grid->dx;
    g.ih[1] = 1.0 / grid->dy;
    g.ih[2] = 1.0 / grid->dz;
    g.gamma = gamma;
    g.alpha = alpha;
    for (int d = 0; d < 3; ++d) g.periodic[d] = bc->face[2 * d] == IGR_BC_PERIODIC;
    const bool split = c->precision == IGR_F32_BF16D;
    c->esize = c->precision == IGR_F64 ? 8 : (c->precision == IGR_F32 || split) ? 4 : 2;   // BF16 and F16: 2
    c->dsize = split ? 2 : c->esize;
    c->ssize = split ? 2 : c->esize;
    c->csize = c->precision == IGR_F64 ? 8 : 4;
    if (c->sigma_block == 0) {
        // Two sweeps per pass halve the sweeps' memory traffic but cost
        // more instructions per sweep.  In FP64 the sweeps are bound by
        // memory at every size.  With FP32 arithmetic the single-sweep
        // kernel wins while one sweep's working set (Sigma in and out, rho
        // or the stored 1/rho, the FP32 source) stays in the last-level
        // cache, whose reuse the two-sweep pass cannot improve on.
        const double rho_bytes = split ? double(c->csize) : double(c->esize);
        const double sweep_bytes = double(g.fs) * (2.0 * c->ssize + rho_bytes + c->csize);
        c->sigma_block = (c->precision == IGR_F64 || sweep_bytes > IGR_LLC_BYTES) ? 2 : 1;
    }

    auto alloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? IGR_ENOMEM : IGR_EHIP,
                                         std::string("hipMalloc: ") + hipGetErrorString(e));
        return IGR_OK;
    };
    int rc = IGR_OK;
    if (hipGetDevice(&c->device) != hipSuccess) rc = fail(IGR_EHIP, "hipGetDevice failed");
    if (!rc) rc = alloc(&c->d_Ua, 5 * field_bytes(c, c->dsize));
    if (!rc) rc = alloc(&c->d_Ub, 5 * field_bytes(c, c->dsize));
    if (!rc) rc = alloc(&c->d_sig2, field_bytes(c, c->ssize));
    if (!rc) rc = alloc(&c->d_b, field_bytes(c, c->csize));
    if (!rc && split) rc = alloc(&c->d_ir, field_bytes(c, c->csize));
    if (!rc && split) rc = alloc(&c->d_Unb, 5 * field_bytes(c, c->esize));
    if (!rc && c->viscous) rc = alloc(&c->d_G, 6 * field_bytes(c, c->csize));
    if (!rc) rc = alloc((void**)&c->d_partial, 5 * RED_BLOCKS * sizeof(double));
    if (!rc) rc = alloc((void**)&c->d_scalars, 8 * sizeof(double));
    if (!rc) rc = alloc((void**)&c->d_flag, sizeof(int));
    if (!rc) {
        // per-block CFL maxima: of the last flux stage (igr_advance), of the
        // first sweep or pass (FP64 igr_step), or of the last viscous
        // launch (igr_advance with viscous terms)
        long long nb = c->precision == IGR_F64         ? flux_blocks<Plain<double>>(c)
                       : c->precision == IGR_F32_BF16D ? flux_blocks<Split>(c)
                                                       : flux_blocks<Plain<float>>(c);
        if (c->precision == IGR_F64 && sweep_speed_slots(c->g) > nb) nb = sweep_speed_slots(c->g);
        if (c->precision == IGR_F64 && pair_speed_slots(c->g) > nb) nb = pair_speed_slots(c->g);
        // with viscous terms: of the last viscous flux-divergence launch
        if (c->viscous) {
            // (the 16-bit forms run the FP32-arithmetic shape)
            const long long nv = c->precision == IGR_F64 ? visc_blocks<Plain<double>>(c) : visc_blocks<Plain<float>>(c);
            if (nv > nb) nb = nv;
        }
        rc = alloc((void**)&c->d_speed, size_t(nb) * sizeof(double));
    }
    if (!rc && !c->patches.empty()) {
        const size_t cols = (size_t)c->ny * c->nz;
        rc = alloc((void**)&c->d_owner, cols * sizeof(int));
        if (!rc) rc = alloc((void**)&c->d_chi, cols * sizeof(double));
        if (!rc) rc = alloc((void**)&c->d_jet, c->patches.size() * 5 * sizeof(double));
        if (!rc) rc = alloc((void**)&c->d_jet0, c->patches.size() * 5 * sizeof(double));
        if (!rc && hipMemset(c->d_jet0, 0, c->patches.size() * 5 * sizeof(double)) != hipSuccess)
            rc = fail(IGR_EHIP, "zero jet table initialisation failed");
        if (!rc) rc = upload_patches(c);
        if (!rc) rc = upload_jets(c, nullptr, true);
    }
    if (!rc) {
        // scratch starts defined: zero states, Sigma copy and source
        if (hipMemset(c->d_Ua, 0, 5 * field_bytes(c, c->dsize)) != hipSuccess ||
            hipMemset(c->d_Ub, 0, 5 * field_bytes(c, c->dsize)) != hipSuccess ||
            hipMemset(c->d_sig2, 0, field_bytes(c, c->ssize)) != hipSuccess ||
            (split && hipMemset(c->d_Unb, 0, 5 * field_bytes(c, c->esize)) != hipSuccess) ||
            (c->viscous && hipMemset(c->d_G, 0, 6 * field_bytes(c, c->csize)) != hipSuccess) ||
            hipMemset(c->d_b, 0, field_bytes(c, c->csize)) != hipSuccess ||
            hipMemset(c->d_flag, 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            rc = fail(IGR_EHIP, "scratch initialisation failed");
    }
    if (rc) {
        release(c);
        return rc;
    }
    *out = c;
    return IGR_OK;
}

int igr_finalize(igr_ctx* ctx) {
    if (!ctx) return IGR_OK;
    const hipError_t e = hipDeviceSynchronize();   // pending work may still use the scratch
    release(ctx);
    if (e != hipSuccess) return fail(IGR_EHIP, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
    return IGR_OK;
}

int igr_field_size(const igr_ctx* ctx, int64_t* elems, int32_t* elem_bytes) {
    if (!ctx) return fail(IGR_EINVAL, "null context");
    if (elems) *elems = ctx->g.fs;
    if (elem_bytes) *elem_bytes = int32_t(ctx->esize);
    return IGR_OK;
}

int igr_get_opts(const igr_ctx* ctx, igr_opts* out) {
    if (!ctx || !out) return fail(IGR_EINVAL, "null argument");
    out->precision = ctx->precision;
    out->order = ctx->order;
    out->nsweeps = ctx->nsweeps;
    out->sigma_block = ctx->sigma_block;
    out->smoother = ctx->smoother;
    out->mu = ctx->mu;
    out->zeta = ctx->zeta;
    return IGR_OK;
}

int igr_set_patch_state(igr_ctx* ctx, int32_t index, const double prim[5], void* stream) {
    if (!ctx || !prim) return fail(IGR_EINVAL, "null argument");
    if (index < 0 || index >= (int)ctx->patches.size()) return fail(IGR_EINVAL, "patch index out of range");
    if (!(prim[0] > 0) || !(prim[4] > 0)) return fail(IGR_EINVAL, "jet needs rho > 0 and p > 0");
    igr_patch& pa = ctx->patches[index];
    pa.rho = prim[0];
    pa.ux = prim[1];
    pa.uy = prim[2];
    pa.uz = prim[3];
    pa.p = prim[4];
    // the new conserved state travels as kernel arguments, ordered on the
    // stream like every other call (work queued before it still reads the
    // old state; no host buffer has to outlive the call)
    const double gm = ctx->g.gamma;
    const double E = pa.p / (gm - 1.0) + 0.5 * pa.rho * (pa.ux * pa.ux + pa.uy * pa.uy + pa.uz * pa.uz);
    hipStream_t s = as_stream(stream);
    k_set_jet<<<1, 64, 0, s>>>(ctx->d_jet, index, pa.rho, pa.rho * pa.ux, pa.rho * pa.uy, pa.rho * pa.uz, E);
    IGR_HIP(hipGetLastError());
    return IGR_OK;
}

int igr_sigma_solve(igr_ctx* ctx, void* U, void* sigma, int32_t nsweeps, double* resid_l2, void* stream) {
    if (!ctx || !U || !sigma) return fail(IGR_EINVAL, "null argument");
    if (nsweeps < 0) return fail(IGR_EINVAL, "nsweeps must be >= 0");
    return DISPATCH(ctx, sigma_t, ctx, U, sigma, nsweeps, resid_l2, as_stream(stream));
}

int igr_rhs(igr_ctx* ctx, void* U, void* sigma, void* rhs, void* stream) {
    if (!ctx || !U || !sigma || !rhs) return fail(IGR_EINVAL, "null argument");
    if (rhs == U || rhs == sigma) return fail(IGR_EINVAL, "rhs must not alias U or sigma");
    return DISPATCH(ctx, rhs_t, ctx, U, sigma, rhs, as_stream(stream));
}

int igr_step(igr_ctx* ctx, void* U, void* sigma, double cfl, double dt_fixed, double* dt_used, void* stream) {
    if (!ctx || !U || !sigma) return fail(IGR_EINVAL, "null argument");
    if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(IGR_EINVAL, "need cfl > 0 or dt_fixed > 0");
    hipStream_t s = as_stream(stream);
    IGR_TRY(DISPATCH(ctx, step_t, ctx, U, sigma, cfl, dt_fixed, s));
    if (dt_used) {
        if (dt_fixed > 0.0) {
            *dt_used = dt_fixed;
        } else {
            IGR_HIP(hipMemcpyAsync(dt_used, ctx->d_scalars, sizeof(double), hipMemcpyDeviceToHost, s));
        }
        return read_flag(ctx, s);
    }
    return IGR_OK;
}

int igr_advance(igr_ctx* ctx, void* U, void* sigma, int32_t nsteps, double cfl, double dt_fixed, double* dt_last,
                void* stream) {
    if (!ctx || !U || !sigma) return fail(IGR_EINVAL, "null argument");
    if (nsteps < 0) return fail(IGR_EINVAL, "nsteps must be >= 0");
    if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(IGR_EINVAL, "need cfl > 0 or dt_fixed > 0");
    hipStream_t s = as_stream(stream);
    IGR_TRY(DISPATCH(ctx, advance_t, ctx, U, sigma, nsteps, cfl, dt_fixed, s));
    if (dt_last) {
        if (dt_fixed > 0.0 || nsteps == 0) {
            *dt_last = dt_fixed > 0.0 ? dt_fixed : 0.0;
        } else {
            IGR_HIP(hipMemcpyAsync(dt_last, ctx->d_scalars, sizeof(double), hipMemcpyDeviceToHost, s));
        }
        return read_flag(ctx, s);
    }
    return IGR_OK;
}

int igr_compute_dt(igr_ctx* ctx, const void* U, double cfl, double* dt, void* stream) {
    if (!ctx || !U || !dt) return fail(IGR_EINVAL, "null argument");
    if (!(cfl > 0.0)) return fail(IGR_EINVAL, "cfl must be > 0");
    hipStream_t s = as_stream(stream);
    IGR_TRY(DISPATCH(ctx, dt_t, ctx, U, cfl, s));
    IGR_HIP(hipMemcpyAsync(dt, ctx->d_scalars, sizeof(double), hipMemcpyDeviceToHost, s));
    return read_flag(ctx, s);
}

int igr_sums(igr_ctx* ctx, const void* U, double out[5], void* stream) {
    if (!ctx || !U || !out) return fail(IGR_EINVAL, "null argument");
    return DISPATCH(ctx, sums_t, ctx, U, out, as_stream(stream));
}

int igr_check(igr_ctx* ctx, void* stream) {
    if (!ctx) return fail(IGR_EINVAL, "null context");
    return read_flag(ctx, as_stream(stream));
}

int igr_timing(igr_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(IGR_EINVAL, "null context");
    if (enable && !ctx->timing) {
        IGR_TRY(collect_timing(ctx));
        for (int k = 0; k < K_COUNT; ++k) {
            ctx->kernel_ms[k] = 0.0;
            ctx->kernel_count[k] = 0;
        }
    }
    ctx->timing = enable != 0;
    return IGR_OK;
}

int igr_kernel_time(igr_ctx* ctx, const char* name, double* ms, int64_t* count) {
    if (!ctx || !name) return fail(IGR_EINVAL, "null argument");
    IGR_TRY(collect_timing(ctx));
    for (int k = 0; k < K_COUNT; ++k) {
        if (std::strcmp(name, kKernelNames[k]) == 0) {
            if (ms) *ms = ctx->kernel_ms[k];
            if (count) *count = ctx->kernel_count[k];
            return IGR_OK;
        }
    }
    return fail(IGR_EINVAL, std::string("unknown kernel name ") + name);
}

int igr_rhs_adjoint(igr_ctx* ctx, void* U, const void* sigma_prev, const void* rhs_bar, const void* sigma_bar,
                    void* U_bar, void* sigma_prev_bar, double* patch_bar, void* stream) {
    if (!ctx || !U || !sigma_prev || !rhs_bar || !sigma_bar || !U_bar || !sigma_prev_bar)
        return fail(IGR_EINVAL, "null argument");
    if (ctx->precision != IGR_F64) return fail(IGR_EUNSUPPORTED, "the adjoint is implemented for IGR_F64");
    if (ctx->smoother != IGR_SMOOTH_JACOBI) return fail(IGR_EUNSUPPORTED, "the adjoint is implemented for Jacobi sweeps");
    hipStream_t s = as_stream(stream);
    IGR_TRY(adjoint_buffers(ctx));
    // inputs may alias outputs: stage them
    double* Lb = abuf(ctx, A_LB);
    double* Sbn = abuf(ctx, A_SBIN);
    IGR_TRY(dcopy(ctx, Lb, (const double*)rhs_bar, 5, s));
    IGR_TRY(dcopy(ctx, Sbn, (const double*)sigma_bar, 1, s));
    std::vector<double> jbar(ctx->patches.size() * 5, 0.0);
    double* Ust = abuf(ctx, A_UST);
    IGR_TRY(dzero(ctx, (double*)U_bar, 5, s));
    IGR_TRY(dzero(ctx, (double*)sigma_prev_bar, 1, s));
    IGR_TRY(stage_adjoint(ctx, (double*)U, (const double*)sigma_prev, Lb, Sbn, Ust, abuf(ctx, A_SBIN), jbar, s));
    IGR_TRY(axpby(ctx, 1.0, Ust, 0.0, (double*)U_bar, 5, s));
    IGR_TRY(axpby(ctx, 1.0, abuf(ctx, A_SBIN), 0.0, (double*)sigma_prev_bar, 1, s));
    IGR_HIP(hipStreamSynchronize(s));
    if (patch_bar) jet_primitive_bar(ctx, jbar, patch_bar);
    return IGR_OK;
}

int igr_step_adjoint(igr_ctx* ctx, void* U_n, const void* sigma_n, double dt, const void* U_bar_np1,
                     const void* sigma_bar_np1, void* U_bar_n, void* sigma_bar_n, double* patch_bar, void* stream) {
    if (!ctx || !U_n || !sigma_n || !U_bar_np1 || !sigma_bar_np1 || !U_bar_n || !sigma_bar_n)
        return fail(IGR_EINVAL, "null argument");
    if (ctx->precision != IGR_F64) return fail(IGR_EUNSUPPORTED, "the adjoint is implemented for IGR_F64");
    if (ctx->smoother != IGR_SMOOTH_JACOBI) return fail(IGR_EUNSUPPORTED, "the adjoint is implemented for Jacobi sweeps");
    if (!(dt > 0.0)) return fail(IGR_EINVAL, "the step adjoint needs a fixed dt > 0");
    hipStream_t s = as_stream(stream);
    IGR_TRY(adjoint_buffers(ctx));
    const int S = ctx->nsweeps;
    double* Un = (double*)U_n;
    double* U1 = abuf(ctx, A_U1);
    double* U2 = abuf(ctx, A_U2);
    double* sig1 = abuf(ctx, A_SIG1);
    double* sig2 = abuf(ctx, A_SIG2);
    double* Ub3 = abuf(ctx, A_UBIN);
    double* Sb3 = abuf(ctx, A_SBIN);
    IGR_TRY(dcopy(ctx, Ub3, (const double*)U_bar_np1, 5, s));
    IGR_TRY(dcopy(ctx, Sb3, (const double*)sigma_bar_np1, 1, s));
    // forward recompute of the stage states and stage warm starts
    IGR_TRY(fill_state_ghosts(ctx, Un, s));
    IGR_TRY(dcopy(ctx, sig1, (const double*)sigma_n, 1, s));
    IGR_TRY(sigma_solve_impl<Plain<double>>(ctx, Un, sig1, S, s));
    IGR_TRY((flux_impl<Plain<double>, MODE_STAGE1>(ctx, Un, nullptr, sig1, nullptr, U1, nullptr, dt, s)));
    if (ctx->viscous) IGR_TRY((viscous_impl<Plain<double>, MODE_STAGE1>(ctx, Un, nullptr, U1, nullptr, dt, s)));
    IGR_TRY(fill_state_ghosts(ctx, U1, s));
    IGR_TRY(dcopy(ctx, sig2, sig1, 1, s));
    IGR_TRY(sigma_solve_impl<Plain<double>>(ctx, U1, sig2, S, s));
    IGR_TRY((flux_impl<Plain<double>, MODE_STAGE2>(ctx, U1, nullptr, sig2, Un, U2, nullptr, dt, s)));
    if (ctx->viscous) IGR_TRY((viscous_impl<Plain<double>, MODE_STAGE2>(ctx, U1, nullptr, U2, nullptr, dt, s)));
    // reverse sweep over the stages
    double* Ubn = abuf(ctx, A_UBN);
    double* Ub1 = abuf(ctx, A_UB1);
    double* Ub2 = abuf(ctx, A_UB2);
    double* Lb = abuf(ctx, A_LB);
    double* Ust = abuf(ctx, A_UST);
    double* sbs = abuf(ctx, A_SBIN);   // running Sigma-bar (stage outputs -> inputs)
    std::vector<double> jbar(ctx->patches.size() * 5, 0.0);
    // stage 3: U3 = Un/3 + 2/3 (U2 + dt L(U2, Sigma2))
    IGR_TRY(axpby(ctx, 1.0 / 3.0, Ub3, 0.0, Ubn, 5, s));
    IGR_TRY(axpby(ctx, 2.0 / 3.0, Ub3, 0.0, Ub2, 5, s));
    IGR_TRY(axpby(ctx, 2.0 / 3.0 * dt, Ub3, 0.0, Lb, 5, s));
    IGR_TRY(stage_adjoint(ctx, U2, sig2, Lb, sbs, Ust, sbs, jbar, s));
    IGR_TRY(axpby(ctx, 1.0, Ust, 1.0, Ub2, 5, s));
    // stage 2: U2 = 3/4 Un + 1/4 (U1 + dt L(U1, Sigma1))
    IGR_TRY(axpby(ctx, 0.75, Ub2, 1.0, Ubn, 5, s));
    IGR_TRY(axpby(ctx, 0.25, Ub2, 0.0, Ub1, 5, s));
    IGR_TRY(axpby(ctx, 0.25 * dt, Ub2, 0.0, Lb, 5, s));
    IGR_TRY(stage_adjoint(ctx, U1, sig1, Lb, sbs, Ust, sbs, jbar, s));
    IGR_TRY(axpby(ctx, 1.0, Ust, 1.0, Ub1, 5, s));
    // stage 1: U1 = Un + dt L(Un, Sigma_n)
    IGR_TRY(axpby(ctx, 1.0, Ub1, 1.0, Ubn, 5, s));
    IGR_TRY(axpby(ctx, dt, Ub1, 0.0, Lb, 5, s));
    IGR_TRY(stage_adjoint(ctx, Un, (const double*)sigma_n, Lb, sbs, Ust, sbs, jbar, s));
    IGR_TRY(axpby(ctx, 1.0, Ust, 1.0, Ubn, 5, s));
    IGR_TRY(dzero(ctx, (double*)U_bar_n, 5, s));
    IGR_TRY(dzero(ctx, (double*)sigma_bar_n, 1, s));
    IGR_TRY(axpby(ctx, 1.0, Ubn, 0.0, (double*)U_bar_n, 5, s));
    IGR_TRY(axpby(ctx, 1.0, sbs, 0.0, (double*)sigma_bar_n, 1, s));
    IGR_HIP(hipStreamSynchronize(s));
    if (patch_bar) jet_primitive_bar(ctx, jbar, patch_bar);
    return IGR_OK;
}


int igr_compute_dt_noalloc(const igr_grid* grid, double gamma, int32_t precision, const void* U, double cfl,
                           double* dt, void* stream) {
    if (!grid || !U || !dt) return fail(IGR_EINVAL, "null argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(IGR_EINVAL, "grid extents must be >= 1");
    if (!(grid->dx > 0) || !(grid->dy > 0) || !(grid->dz > 0)) return fail(IGR_EINVAL, "spacings must be > 0");
    if (!(gamma > 1.0)) return fail(IGR_EINVAL, "gamma must be > 1");
    if (!(cfl > 0.0)) return fail(IGR_EINVAL, "cfl must be > 0");
    if (precision != IGR_F64 && precision != IGR_F32 && precision != IGR_BF16_F32 && precision != IGR_F16_F32 &&
        precision != IGR_F32_BF16D)
        return fail(IGR_EINVAL, "unknown precision");
    const long long px = grid->nx + 2 * G, py = grid->ny + 2 * G, pz = grid->nz + 2 * G;
    if (px * py > 0x7fffffffLL) return fail(IGR_EINVAL, "x-y plane too large");
    // the reduction runs on a fixed grid of RED_BLOCKS blocks whatever the
    // extents, so its partials always fit the scratch
    if (kNoAllocFlagOff + sizeof(int) > kNoAllocBytes) return fail(IGR_EINVAL, "reduction exceeds the scratch");
    Geom g{};
    g.n[0] = grid->nx;
    g.n[1] = grid->ny;
    g.n[2] = grid->nz;
    g.st[0] = 1;
    g.st[1] = int(px);
    g.st[2] = int(px * py);
    g.fs = px * py * pz;
    g.ih[0] = 1.0 / grid->dx;
    g.ih[1] = 1.0 / grid->dy;
    g.ih[2] = 1.0 / grid->dz;
    g.gamma = gamma;
    unsigned char* base = nullptr;
    IGR_TRY(noalloc_scratch(&base));
    double* partial = reinterpret_cast<double*>(base + kNoAllocPartialOff);
    double* result = reinterpret_cast<double*>(base + kNoAllocResultOff);
    int* flag = reinterpret_cast<int*>(base + kNoAllocFlagOff);
    hipStream_t s = as_stream(stream);
    IGR_TRY(precision == IGR_F64   ? dt_noalloc_t<double>(g, U, partial, result, flag, cfl, s)
            : (precision == IGR_F32 || precision == IGR_F32_BF16D) ? dt_noalloc_t<float>(g, U, partial, result, flag, cfl, s)
            : precision == IGR_F16_F32 ? dt_noalloc_t<f16>(g, U, partial, result, flag, cfl, s)
                                       : dt_noalloc_t<bf16>(g, U, partial, result, flag, cfl, s));
    int bad = 0;
    IGR_HIP(hipMemcpyAsync(dt, result, sizeof(double), hipMemcpyDeviceToHost, s));
    IGR_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    IGR_HIP(hipStreamSynchronize(s));
    if (bad) return fail(IGR_ENONFINITE, "a kernel saw rho <= 0, p <= 0 or a non-finite value");
    return IGR_OK;
}

}  // extern "C"
