// Host orchestration and the C ABI of the nested block solver.
//
// One Newton step = tangent assembly (Sec. 2.5, steps 6 and 8), per-step
// preconditioner set-up, and FGMRES(m) (Sec. 3) right-preconditioned by the
// Schur complement reduction P_SCR (Algorithm 3) whose Schur solve uses the
// matrix-free action of Algorithm 2.  All vector, matrix and reduction work
// runs in HIP kernels; the host drives the Krylov loops and reads one status
// record per Krylov iteration for the stopping test.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <type_traits>

#include "kernels.h"

using namespace ns;

namespace {

thread_local std::string g_create_err;

struct Fail {
    ns_status st;
    std::string msg;
};

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess)                                                                      \
            throw Fail{NS_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_) + " (line " +     \
                                       std::to_string(__LINE__) + ")"};                            \
    } while (0)

inline void check_launch() { HIPCHK(hipGetLastError()); }

template <typename T>
inline T* as(double* p) {
    return reinterpret_cast<T*>(p);
}

int dflt(int v, int d) { return v > 0 ? v : d; }
double dfltd(double v, double d) { return v > 0 ? v : d; }
// AMG smoother defaults: Chebyshev degree 2 on [lambda/10, lambda]
constexpr int kDefaultChebDegree = 2;
constexpr double kDefaultChebRatio = 10.0;
// V-cycle iterations per application of P_S.  More than one helps on small
// meshes but the stationary V-cycle iteration on S_hat can diverge (observed
// on the 1e6-node Y-bifurcation), so the default is a single V-cycle.
constexpr int kDefaultCyclesS = 1;
// Scaling of the coarse-grid correction of each hierarchy (1: the plain
// Galerkin correction).
constexpr double kDefaultCcScaleA = 1.0;
constexpr double kDefaultCcScaleS = 1.0;
constexpr double kXcdMaxXBytes = 8.0e6;

// ---------------------------------------------------------------------------
// workspace layout (measured with a null base, then applied to the real one)
// ---------------------------------------------------------------------------

template <typename T>
T* up(Arena& A, const std::vector<T>& v) {
    return A.take<T>(std::max<size_t>(v.size(), 1));
}

void layout(ns_ctx* c, Arena& A) {
    const Symbolic& S = c->sym;
    const int N = S.N;
    const int64_t nnzb = S.g.nnz();
    const int64_t nS = S.shat.nnz();
    const int nslot = (int)S.onode.size();
    const int NO = S.n_out;
    c->d_rp = up(A, S.g.rp);
    c->d_col = up(A, S.g.col);
    c->d_dcol = S.dcol.empty() ? nullptr : up(A, S.dcol);
    c->d_dcol_ell = S.dcol_ell.empty() ? nullptr : up(A, S.dcol_ell);
    c->d_diag = up(A, S.diag_pos);
    c->d_rowof = up(A, S.row_of);
    c->d_tmap = up(A, S.tmap);
    c->d_tets = up(A, S.tets);
    c->d_emap = up(A, S.emap);
    c->d_faces = up(A, S.faces);
    c->d_fmap = up(A, S.fmap);
    c->d_fslot = up(A, S.fslot);
    c->d_face_out = up(A, S.face_out);
    c->d_onode = up(A, S.onode);
    c->d_oid = up(A, S.oid);
    c->d_slot_of = up(A, S.slot_of);
    c->d_optr = up(A, S.optr);
    c->d_srp = up(A, S.shat.rp);
    c->d_scol = up(A, S.shat.col);
    c->d_mask = A.take<uint8_t>((size_t)N * 4);
    c->d_xyz = A.take<double>((size_t)N * 3);
    c->d_a_raw = A.take<double>(std::max(1, nslot * 3));
    c->d_a_msk = A.take<double>(std::max(1, nslot * 3));
    c->d_a_msk32 = A.take<float>(std::max(1, nslot * 3));
    c->d_aos = A.take<double>((size_t)nnzb * 16);
    c->d_res = A.take<double>((size_t)N * 4);
    c->d_ck = A.take<double>(std::max(1, NO));
    c->d_ck32 = A.take<float>(std::max(1, NO));
    c->d_s = A.take<double>(std::max(1, NO));
    c->d_s2 = A.take<double>(std::max(1, NO));
    c->d_R = A.take<double>(std::max(1, NO));
    c->d_Pn = A.take<double>(std::max(1, NO));
    c->d_Q = A.take<double>(std::max(1, NO));
    c->d_grad = A.take<double>(std::max(1, NO));
    c->d_Paf = A.take<double>(std::max(1, NO));
    const int mo = dflt(c->opts.max_m, 200), ma = dflt(c->opts.max_m_A, 200), ms = dflt(c->opts.max_m_S, 200);
    const int mmax = std::max(mo, std::max(ma, ms));
    c->d_red = A.take<double>((size_t)(mmax + 4) * kMaxRedBlocks);

    // AMG patterns (shared by the forward and transposed systems)
    const int L = (int)S.lv.size();
    for (int s = 0; s < 2; ++s) {
        c->sys[s].A.assign(L, AmgLevelDev{});
        c->sys[s].S.assign(L, AmgLevelDev{});
    }
    for (int l = 0; l < L; ++l) {
        const AmgLevelSym& ls = S.lv[l];
        AmgLevelDev& a = c->sys[0].A[l];
        AmgLevelDev& sd = c->sys[0].S[l];
        a.n = sd.n = ls.n;
        a.bs = 3;
        sd.bs = 1;
        a.nnz = ls.a.nnz();
        sd.nnz = ls.s.nnz();
        if (l == 0) {
            a.rp = c->d_rp;
            a.col = c->d_col;
            sd.rp = c->d_srp;
            sd.col = c->d_scol;
        } else {
            a.rp = up(A, ls.a.rp);
            a.col = up(A, ls.a.col);
            sd.rp = up(A, ls.s.rp);
            sd.col = up(A, ls.s.col);
            a.gptr = up(A, ls.gptr);
            a.gidx = up(A, ls.gidx);
            a.qrow = up(A, ls.a_qrow);
            sd.gptr = up(A, ls.sgptr);
            sd.gidx = up(A, ls.sgidx);
            sd.qrow = a.qrow;  // unused for S
        }
        if (l + 1 < L) {
            a.agg = sd.agg = up(A, ls.agg);
            a.aptr = sd.aptr = up(A, ls.aptr);
            a.anodes = sd.anodes = up(A, ls.anodes);
        }
        for (AmgLevelDev* d : {&a, &sd}) {
            const int64_t nv = (int64_t)d->n * d->bs;
            d->x0 = A.take<double>(nv);
            d->x1 = A.take<double>(nv);
            d->d = A.take<double>(nv);
            d->r = A.take<double>(nv);
            d->b = A.take<double>(nv);
        }
        c->sys[1].A[l] = a;
        c->sys[1].S[l] = sd;
    }
    // numeric values per system
    for (int s = 0; s < 2; ++s) {
        SystemDev& y = c->sys[s];
        y.V64 = A.take<double>((size_t)nnzb * 16);
        // FP32 planes: the node graph's layout or the fixed-width rows (chosen at bind)
        y.V32 = A.take<float>((size_t)std::max<int64_t>(nnzb, (int64_t)N * S.ell) * 16);
        y.dK64 = A.take<double>((size_t)N * 3);
        y.diagA64 = A.take<double>((size_t)N * 3);
        y.dinvA64 = A.take<double>((size_t)N * 3);
        y.dK32 = A.take<float>((size_t)N * 3);
        y.dinvA32 = A.take<float>((size_t)N * 3);
        y.shat64 = A.take<double>(nS);
        y.shat32 = A.take<float>(nS);
        for (int l = 0; l < L; ++l) {
            for (int h = 0; h < 2; ++h) {
                AmgLevelDev& d = h == 0 ? y.A[l] : y.S[l];
                const int64_t nv = (int64_t)d.n * d.bs;
                if (l == 0) {
                    if (h == 0) {
                        d.v64 = y.V64;
                        d.v32 = y.V32;
                        d.rstride = 4 * nnzb;
                        d.cstride = nnzb;
                        d.dinv64 = y.dinvA64;
                        d.dinv32 = y.dinvA32;
                        d.dextra64 = y.dK64;
                        d.dextra32 = y.dK32;
                    } else {
                        d.v64 = y.shat64;
                        d.v32 = y.shat32;
                        d.dinv64 = A.take<double>(nv);
                        d.dinv32 = A.take<float>(nv);
                    }
                } else {
                    d.v64 = A.take<double>((size_t)d.nnz * d.bs * d.bs);
                    d.v32 = A.take<float>((size_t)d.nnz * d.bs * d.bs);
                    d.rstride = d.bs * d.nnz;
                    d.cstride = d.nnz;
                    d.dinv64 = A.take<double>(nv);
                    d.dinv32 = A.take<float>(nv);
                }
                if (l == L - 1) {
                    d.inv = A.take<double>((size_t)nv * nv);
                    d.work = A.take<double>((size_t)nv * 4 * nv);  // two halves of [M | I]
                } else {
                    d.coef64 = A.take<double>(kCoefLen);
                    d.coef32 = A.take<float>(kCoefLen);
                }
            }
        }
    }
    // Krylov workspaces
    auto kry = [&](KrylovWs& k, int m, int64_t n, bool outer) {
        k.m = m;
        k.n = n;
        k.ld = (n + 63) / 64 * 64;
        k.V = A.take<double>((size_t)(m + 1) * k.ld);
        k.Z = outer ? A.take<double>((size_t)m * k.ld) : nullptr;
        k.tmp = A.take<double>(n);
        k.H = A.take<double>((size_t)(m + 1) * m);
        k.cs = A.take<double>(m);
        k.sn = A.take<double>(m);
        k.g = A.take<double>(m + 1);
        k.y = A.take<double>(m);
        k.h = A.take<double>(2 * (size_t)(m + 2));
        k.status = A.take<double>(8);
    };
    kry(c->kw_out, mo, 4 * (int64_t)N, true);
    kry(c->kw_A, ma, 3 * (int64_t)N, false);
    kry(c->kw_S, ms, (int64_t)N, false);
    c->t_s = A.take<double>(4 * (size_t)N);
    c->t_yhat = A.take<double>(3 * (size_t)N);
    c->t_tp = A.take<double>(N);
    c->t_yp = A.take<double>(4 * (size_t)N);
    c->t_tv = A.take<double>(3 * (size_t)N);
    c->t_yv = A.take<double>(3 * (size_t)N);
    c->t_xhat = A.take<double>(N);
    c->t_xbar = A.take<double>(3 * (size_t)N);
    c->t_xt = A.take<double>(3 * (size_t)N);
    c->t_sf = A.take<double>(4 * (size_t)N);
    c->t_ps = A.take<double>(2 * (size_t)N);
    c->nt_yaf = A.take<double>(4 * (size_t)N);
    c->nt_ydam = A.take<double>(4 * (size_t)N);
    c->nt_rhs = A.take<double>(4 * (size_t)N);
    c->nt_dx = A.take<double>(4 * (size_t)N);
    c->nt_scal = A.take<double>(8);
    c->d_bnd = A.take<double>(3 * 2 * std::max<size_t>(S.lv.size(), 1));
    c->t_r4 = A.take<double>(4 * (size_t)N);
    A.take<char>(256);
}

template <typename T>
void h2d(T* d, const std::vector<T>& v, hipStream_t st) {
    if (!v.empty()) HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// ---------------------------------------------------------------------------
// Kernel timing: bracket launches of selected classes with event pairs
// ---------------------------------------------------------------------------

constexpr size_t kTimingPairs = 65536;

template <typename F>
void timed(ns_ctx* c, int cls, double bytes, hipStream_t st, F&& launch) {
    const size_t used = c->kt_pending.size();
    if (!(c->kt_mask & (1 << cls)) || used >= kTimingPairs || c->kt_seen[cls]++ % (uint64_t)c->kt_period != 0) {
        launch();
        return;
    }
    while (c->kt_ev.size() < 2 * (used + 1)) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->kt_ev.push_back(e);
    }
    // the launch itself records the pair at the kernel's start and end
    set_launch_events(c->kt_ev[2 * used], c->kt_ev[2 * used + 1]);
    launch();
    if (launch_events_pending()) {  // no timed kernel was launched: drop the sample
        set_launch_events(nullptr, nullptr);
        return;
    }
    c->kt_pending.emplace_back(cls, bytes);
}

// after the stream has been synchronised: fold the recorded pairs into the totals
void timing_collect(ns_ctx* c) {
    for (size_t i = 0; i < c->kt_pending.size(); ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->kt_ev[2 * i], c->kt_ev[2 * i + 1]));
        const int cls = c->kt_pending[i].first;
        c->kt_acc[cls][0] += 1.0;
        c->kt_acc[cls][1] += ms;
        c->kt_acc[cls][2] += c->kt_pending[i].second;
    }
    c->kt_pending.clear();
}

// ---------------------------------------------------------------------------
// Schedule of Krylov iteration counts
// ---------------------------------------------------------------------------

struct Sched {
    const int32_t* replay = nullptr;
    int replay_len = 0;
    std::vector<int32_t> log;
    int begin(int& forced) {
        const int idx = (int)log.size();
        log.push_back(0);
        forced = -1;
        if (replay) {
            if (idx >= replay_len) throw Fail{NS_ERR_ARG, "iteration schedule shorter than the solve"};
            forced = replay[idx];
        }
        return idx;
    }
    void end(int idx, int count) { log[idx] = count; }
};

// ---------------------------------------------------------------------------
// The solver for one system (forward or transposed), precision T inside P_SCR
// ---------------------------------------------------------------------------

template <typename T>
struct Typed;
template <>
struct Typed<double> {
    static const double* V(const SystemDev& y) { return y.V64; }
    static const double* lv(const AmgLevelDev& d) { return d.v64; }
    static const double* dinv(const AmgLevelDev& d) { return d.dinv64; }
    static const double* dextra(const AmgLevelDev& d) { return d.dextra64; }
    static const double* coef(const AmgLevelDev& d) { return d.coef64; }
    static const double* dinvA(const SystemDev& y) { return y.dinvA64; }
    static const double* amsk(const ns_ctx* c) { return c->d_a_msk; }
    static const double* ck(const ns_ctx* c) { return c->d_ck; }
};
template <>
struct Typed<float> {
    static const float* V(const SystemDev& y) { return y.V32; }
    static const float* lv(const AmgLevelDev& d) { return d.v32; }
    static const float* dinv(const AmgLevelDev& d) { return d.dinv32; }
    static const float* dextra(const AmgLevelDev& d) { return d.dextra32; }
    static const float* coef(const AmgLevelDev& d) { return d.coef32; }
    static const float* dinvA(const SystemDev& y) { return y.dinvA32; }
    static const float* amsk(const ns_ctx* c) { return c->d_a_msk32; }
    static const float* ck(const ns_ctx* c) { return c->d_ck32; }
};

struct Ctl {
    ns_ctx* c;
    SystemDev* sy;
    ns_solve_opts o;
    Sched sc;
    hipStream_t st;
    ns_stats stats{};
};

void read_status(ns_ctx* c, const double* d_status, int n, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(c->h_pinned, d_status, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
}

// host-mapped scalar slots written by kernels: [0..1] Arnoldi status, [8] norms
// [9 + kind] initial residual norm of a left GMRES call of that kind
constexpr int kMapStatus = 0, kMapNorm = 8, kMapNorm0 = 9, kMapSeq = 32;
// longest poll of a step's status before falling back to the event wait
constexpr int kStatusPollMs = 50;
// graph kinds of Arnoldi steps (one mapped initial-norm slot each)
constexpr int kKindA = 0, kKindS = 1, kKindOuter = 2, kKindShat = 3, kKindInner = 4, kKindSetup = 5;
// meshes up to this many nodes replay captured graphs by default
constexpr int kGraphMaxNodes = 1024;
// finest A levels from this many rows add the prolongated correction in a pass
// of its own (NS_PROLONG_PASS=0/1, read at bind, forces the fused step or the pass)
constexpr int kProlongPassRows = 500000;
// lanes per row of the factored S_hat passes: 4, a typical row in one trip of
// four blocks per lane (both passes together on the 4e6-node
// contraction-expansion: 500 us with 4 lanes, 545 with 8, 721 with 16)
constexpr int kSfactLanes = 4;

// trip of the 4- and 8-lane row walks: by mean row length, or as forced at
// bind (NS_ROW_UNROLL)
inline int unroll_of(const ns_ctx* c, int64_t nnz, int n) {
    return c->unroll_mode > 0 ? c->unroll_mode : unroll_for(nnz, n);
}
// 16-bit column offsets of the node graph for the finest-level products, when
// the numbering allows them (NS_COL16=0 at bind keeps the 32-bit columns)
inline const int16_t* dcol_of(const ns_ctx* c) { return c->col16 ? c->d_dcol : nullptr; }
// bytes of one column index of the node graph as the finest-level products read it
inline double col_bytes(const ns_ctx* c) { return c->col16 ? 2.0 : 4.0; }

template <typename T>
double dev_norm(ns_ctx* c, int64_t n, const T* x, double* slot, hipStream_t st) {
    norm2<T>(n, x, slot, c->d_red, st, c->d_mapped + kMapNorm);
    check_launch();
    HIPCHK(hipStreamSynchronize(st));
    return static_cast<volatile double*>(c->h_mapped)[kMapNorm];
}

// Launch the executable graph cached under `key` on `st`; the first time,
// capture `body` on `st` into it (thread-local capture, so only this thread's
// calls are restricted).  The bodies record no memset nodes.
template <typename F>
void launch_cached(ns_ctx* c, const ns_ctx::GraphKey& key, hipStream_t st, F&& body) {
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        try {
            body();
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(st, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamEndCapture(st, &g));
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        it = c->graphs.emplace(key, ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, st));
}

// Run one Arnoldi-step body, captured once into a HIP graph per
// (kind, system, precision, P_A, Chebyshev degree, j) and replayed afterwards.
// Every pointer and size the body uses is fixed for the context, and the
// numeric set-up reaches the kernels through device memory, so a graph stays
// valid across tangents.  Kernel timing runs the body eagerly.
template <typename F>
void run_step(ns_ctx* c, const Ctl& K, int kind, int j, F&& body) {
    if (!c->use_graphs || c->kt_mask) {
        body();
        return;
    }
    const int sys = K.sy == &c->sys[0] ? 0 : 1;
    const int degA = dflt(K.o.cheb_degree, kDefaultChebDegree);
    const int cycles = dflt(K.o.cycles_S, kDefaultCyclesS) + 16 * dflt(K.o.cycle_index_S, 1) +
                       256 * dflt(K.o.cycle_index_A, 1);
    const ns_ctx::GraphKey key(kind, sys, K.o.precision, K.o.pc_A, K.o.pc_I, degA, dflt(K.o.cheb_degree_S, degA),
                               cycles, j);
    launch_cached(c, key, K.st, body);
}

// Run one chain of the per-step set-up on stream `st`, captured once per
// (system, chain) and replayed for every later tangent: queued kernel by
// kernel, the set-up's ~300 launches keep the host busier than the device,
// and a replayed chain costs one graph launch.  The chains' pointers and
// sizes are fixed for the context and their inputs are in device memory.
template <typename F>
void run_chain(ns_ctx* c, int sys, int chain, hipStream_t st, F&& body) {
    if (!c->use_graphs) {
        body();
        return;
    }
    launch_cached(c, ns_ctx::GraphKey(kKindSetup, sys, 0, 0, 0, 0, 0, 0, chain), st, body);
}

template <typename T>
void cgs2_launch(ns_ctx* c, KrylovWs& kw, int64_t n, int j, T* V, hipStream_t st, int slot = 0) {
    GivensArgs ga;
    ga.j = j;
    ga.ldh = kw.m + 1;
    ga.h1 = kw.h;
    ga.h2 = kw.h + (kw.m + 2);
    ga.H = kw.H;
    ga.cs = kw.cs;
    ga.sn = kw.sn;
    ga.g = kw.g;
    ga.status = kw.status;
    ga.hstatus = c->d_mapped + kMapStatus + 2 * slot;
    // the step number lets the host read the status as soon as the Givens
    // update has stored it; a captured step would replay a fixed number, so
    // graphs leave it out and their status is read after the step's event
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusNone) {
        ga.hseq = reinterpret_cast<unsigned long long*>(c->d_mapped + kMapSeq + slot);
        ga.seq = ++c->step_seq;
        c->slot_seq[slot] = ga.seq;
    } else {
        c->slot_seq[slot] = 0;
    }
    // algorithmic bytes of the four kernels with k = j + 1 basis vectors: pass-1
    // dots (k + 1 vectors read), pass-1 update and pass-2 dots (2k + 2 read, 1
    // written; k + 1 read when k <= kOrthFuseMax, single pass), pass-2 update
    // (k + 1 read, 1 written), normalisation (1 + 1)
    const int k = j + 1;
    const double bytes = (k <= kOrthFuseMax ? 3.0 * k + 7.0 : 4.0 * k + 8.0) * (double)n * sizeof(T);
    timed(c, NS_KT_CGS2, bytes, st, [&] {
        arnoldi_cgs2<T>(n, j, V, kw.ld, V + (int64_t)(j + 1) * kw.ld, kw.h, kw.h + (kw.m + 2), ga, c->d_red, st);
    });
    check_launch();
}

void read_step_status(ns_ctx* c, KrylovWs& kw, hipStream_t st, double& resid, bool& bd, hipEvent_t ev = nullptr,
                      int slot = 0, bool check = true) {
    // The step's Givens update stores the status and then its step number in
    // mapped host memory: poll for the number (the rest of the step's last
    // kernel keeps running, and later launches queue behind it), for at most
    // kStatusPollMs, then wait for the step's event or the stream as usual.
    bool seen = false;
    const unsigned long long want = c->slot_seq[slot];
    if (want) {
        const volatile unsigned long long* hs =
            reinterpret_cast<const volatile unsigned long long*>(c->h_mapped + kMapSeq + slot);
        const auto t0 = std::chrono::steady_clock::now();
        for (unsigned it = 0;; ++it) {
            if (*hs == want) {
                seen = true;
                break;
            }
            if ((it & 1023u) == 1023u &&
                std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(kStatusPollMs))
                break;
        }
        std::atomic_thread_fence(std::memory_order_acquire);
    }
    if (!seen) {
        if (ev)
            HIPCHK(hipEventSynchronize(ev));
        else
            HIPCHK(hipStreamSynchronize(st));
    }
    const volatile double* h = c->h_mapped + kMapStatus + 2 * slot;
    resid = h[0];
    bd = h[1] != 0.0;
    if (check && !std::isfinite(resid)) throw Fail{NS_ERR_NAN, "residual estimate is not finite"};
}

// Left-preconditioned GMRES(m) for M x = b from x = 0 (Sec. 3.1; stopping on
// the preconditioned residual relative to ||P^{-1} b||).
// kind: graph kind of the Arnoldi step; m_capturable: applyM launches kernels
// only (no host synchronisation), so the whole step is one graph.
// stepM / stepP (optional): the operator and preconditioner as used inside an
// Arnoldi step, where stepM may already perform the preconditioner's first
// smoothing step on its output (the start and restart residuals use applyM
// and applyP); with step_fused, stepM alone computes P^{-1} M v.
template <typename T>
int gmres_left(Ctl& K, KrylovWs& kw, int64_t n, const std::function<void(const T*, T*)>& applyM,
               const std::function<void(const T*, T*)>& applyP, const T* b, T* x, double rtol, int m, int nmax,
               int kind, bool m_capturable, const std::function<void(const T*, T*)>& stepM = {},
               const std::function<void(const T*, T*)>& stepP = {}, bool step_fused = false) {
    const auto& sM = stepM ? stepM : applyM;
    const auto& sP = stepP ? stepP : applyP;
    ns_ctx* c = K.c;
    hipStream_t st = K.st;
    int forced;
    const int idx = K.sc.begin(forced);
    T* V = as<T>(kw.V);
    T* tmp = as<T>(kw.tmp);
    int total = 0;
    applyP(b, V);
    if (forced == 0) {
        fill<T>(n, T(0), x, st);
        K.sc.end(idx, 0);
        return 0;
    }
    // ||P^{-1} b|| stays on the device (status[4], used by the first cycle) and
    // reaches the host through a mapped slot of its own, read together with
    // the first step's status: no host round trip before the first step.
    volatile double* hnorm0 = c->h_mapped + kMapNorm0 + kind;
    norm2<T>(n, V, kw.status + 4, c->d_red, st, c->d_mapped + kMapNorm0 + kind);
    check_launch();
    double beta0 = -1.0, tol = 0.0;  // known after the first status read
    double beta = -1.0;
    bool first = true;
    bool zero_rhs = false;
    while (true) {
        start_cycle<T>(n, V, kw.status + 4, kw.g, m + 1, st);
        int k = 0;
        bool finished = false;
        // Steps of a capturable operator are queued one ahead of the status
        // read (status slot and event alternate with j), unless the residual
        // history predicts convergence at the current step.
        int launched = 0;
        double r_prev = beta, r_prev2 = -1.0;
        auto enqueue = [&](int jj) {
            T* vj = V + (int64_t)jj * kw.ld;
            T* vn = V + (int64_t)(jj + 1) * kw.ld;
            run_step(c, K, kind, jj, [&] {
                if (step_fused) {
                    sM(vj, vn);  // stepM already applies the preconditioner
                } else {
                    sM(vj, tmp);
                    sP(tmp, vn);
                }
                cgs2_launch<T>(c, kw, n, jj, V, st, jj & 1);
            });
            HIPCHK(hipEventRecord(c->step_ev[jj & 1], st));
            launched = jj + 1;
        };
        for (int j = 0; j < m; ++j) {
            double resid;
            bool bd;
            if (m_capturable) {
                if (launched == j) enqueue(j);
                bool ahead = (j + 1 < m) && (total + 2 <= nmax) && (forced < 0 || total + 2 <= forced);
                if (ahead && forced < 0) {
                    if (beta0 < 0.0) {
                        ahead = 0.5 > 2.0 * rtol;  // first step: assume a halving
                    } else {
                        const double ratio = r_prev2 > 0.0 ? r_prev / r_prev2 : 0.5;
                        ahead = r_prev * ratio > 2.0 * tol;
                    }
                }
                if (ahead) enqueue(j + 1);
                read_step_status(c, kw, st, resid, bd, c->step_ev[j & 1], j & 1, false);
            } else {
                sM(V + (int64_t)j * kw.ld, step_fused ? V + (int64_t)(j + 1) * kw.ld : tmp);
                run_step(c, K, kind, j, [&] {
                    if (!step_fused) sP(tmp, V + (int64_t)(j + 1) * kw.ld);
                    cgs2_launch<T>(c, kw, n, j, V, st);
                });
                read_step_status(c, kw, st, resid, bd, nullptr, 0, false);
            }
            if (beta0 < 0.0) {
                beta0 = *hnorm0;
                if (!std::isfinite(beta0)) throw Fail{NS_ERR_NAN, "residual norm is not finite"};
                if (beta0 == 0.0) {
                    zero_rhs = true;
                    break;
                }
                tol = std::max(rtol * beta0, K.o.atol);
                beta = beta0;
                r_prev = beta0;
            }
            if (!std::isfinite(resid)) throw Fail{NS_ERR_NAN, "residual estimate is not finite"};
            r_prev2 = r_prev;
            r_prev = resid;
            ++total;
            k = j + 1;
            const bool done = forced >= 0 ? total >= forced : resid <= tol;
            if (done || bd || total >= nmax) {
                finished = true;
                break;
            }
        }
        if (zero_rhs) {
            // P^{-1} b = 0: the steps already queued ran on a zero basis and
            // are discarded
            fill<T>(n, T(0), x, st);
            check_launch();
            break;
        }
        backsolve(k, kw.m + 1, kw.H, kw.g, kw.y, st);  // H is stored with the workspace leading dimension
        combine<T, T>(n, k, V, kw.ld, kw.y, x, !first, st);
        check_launch();
        first = false;
        if (finished) break;
        // restart: r = P (b - M x)
        applyM(x, tmp);
        axpby<T>(n, T(-1), tmp, T(1), b, tmp, st);
        applyP(tmp, V);
        beta = dev_norm<T>(c, n, V, kw.status + 4, st);
        if (beta == 0.0 || (forced < 0 && beta <= tol)) break;
    }
    K.sc.end(idx, total);
    return total;
}

template <typename T>
struct Nested {
    Ctl& K;
    ns_ctx* c;
    SystemDev& sy;
    int N;
    int64_t nnzb;
    Nested(Ctl& k) : K(k), c(k.c), sy(*k.sy), N(k.c->sym.N), nnzb(k.c->sym.g.nnz()) {}

    const T* V() const { return Typed<T>::V(sy); }
    // FP32 planes in the fixed-width row layout (chosen at bind): plane
    // stride N*ell, slot l of row i at i*ell + l, columns as 16-bit offsets
    bool ell_planes() const { return sizeof(T) == 4 && c->ell32; }
    int ell() const { return ell_planes() ? c->sym.ell : 0; }
    int64_t plane() const { return ell_planes() ? (int64_t)N * c->sym.ell : nnzb; }
    const int16_t* dcol_planes() const { return ell_planes() ? c->d_dcol_ell : dcol_of(c); }
    // XCD-contiguous row ranges pay while a row range's share of the gathered
    // vector stays L2-resident: on when the gathered vector (n*bc values) is
    // at most kXcdMaxXBytes (measured: +15 % on the 2e5-node pipe, -5 % on the
    // 2e6-node pipe); NS_XCD_ROWS=0/1 forces it off/on.
    int xcd_rows(int64_t n, int bc) const {
        if (c->xcd_mode >= 0) return c->xcd_mode;
        return (double)n * bc * sizeof(T) <= kXcdMaxXBytes ? 1 : 0;
    }
    BlockOp<T> op(int r0, int c0) const {
        BlockOp<T> M;
        M.n = N;
        M.rp = c->d_rp;
        M.col = c->d_col;
        M.dcol = dcol_planes();
        M.ell = ell();
        M.v = V() + (4 * r0 + c0) * plane();
        M.rs = 4 * plane();
        M.cs = plane();
        M.lanes = lanes_for(nnzb, N, 3);
        // The thin operators move fewer bytes per block, so fewer lanes per
        // row (more rows, more loads in flight per wave) pay: C (3 values and a
        // 3-wide gather per block) 8 lanes, B and D (one gathered value per
        // block) 4 lanes.  Measured on the 4e6-node contraction-expansion
        // against 16 lanes: C 288 against 386 us, B 268 against 369 us, D 157
        // against 298 us; the 3x3 A operator is fastest with 16 (487 against
        // 533 us with 8 and 556 us with 4).
        if (M.lanes == 16 && (r0 == 3 || c0 == 3)) M.lanes = c0 == 3 ? 4 : 8;
        M.unroll = unroll_of(c, nnzb, N);
        M.xcd = xcd_rows(N, c0 == 3 ? 1 : 3);
        return M;
    }
    BlockOp<T> level_op(const AmgLevelDev& d) const {
        BlockOp<T> M;
        M.n = d.n;
        M.rp = d.rp;
        M.col = d.col;
        if (d.col == c->d_col) M.dcol = dcol_of(c);
        M.v = Typed<T>::lv(d);
        M.rs = d.rstride;
        M.cs = d.cstride;
        if (M.v == V()) {  // the finest A level shares the operator's planes
            M.dcol = dcol_planes();
            M.ell = ell();
            M.rs = 4 * plane();
            M.cs = plane();
        }
        M.dextra = Typed<T>::dextra(d);
        M.lanes = lanes_for(d.nnz, d.n, d.bs);
        M.unroll = unroll_of(c, d.nnz, d.n);
        M.xcd = xcd_rows(d.n, d.bs);
        return M;
    }
    // Factored S_hat application (both passes), timed as one class.
    // Algorithmic bytes: pass 1 reads the three B planes and the column
    // indices, row pointers, x, diag(A)^-1 (and the aggregate map with the
    // coarse correction) and writes t (4 per node); pass 2 reads the three C
    // planes, the D plane, columns, row pointers, t and writes y, plus the
    // Chebyshev operands (b, dinv, d) when smoothing.
    void sfact(const T* x, const int32_t* agg, const T* ec, T* y, T alpha, const T* z, T beta, const T* b,
               const T* dinv, const T* coef, int step, T* d) {
        const double sz = sizeof(T), n = N;
        double bytes = (double)nnzb * (7 * sz + 2 * col_bytes(c)) + 8.0 * (n + 1) + n * sz * (1 + 3 + 4) +
                       n * sz * (4 + 1);
        if (coef) bytes += n * sz * (step != 0 ? 4 : 3);
        else if (z) bytes += n * sz;
        if (agg) bytes += n * (4 + sz);
        timed(c, NS_KT_SFACT, bytes, K.st, [&] {
            shat_factored<T>(N, c->d_rp, c->d_col, dcol_planes(), ell(), V(), plane(), Typed<T>::dinvA(sy), x,
                             agg, ec, as<T>(c->t_sf), y, alpha, z, beta, b, dinv, coef, step, d, xcd_rows(N, 1),
                             kSfactLanes, K.st);
        });
    }
    RankOne<T> rank_one() const {
        RankOne<T> r;
        if (c->sym.n_out == 0) return r;
        r.slot_of = c->d_slot_of;
        r.oid = c->d_oid;
        r.aval = Typed<T>::amsk(c);
        r.s = as<T>(c->d_s);
        return r;
    }
    // first Chebyshev step of the V-cycle on level 0 of H, for fusing into the
    // operator that produces the V-cycle's right-hand side
    FirstStep<T> first_step(std::vector<AmgLevelDev>& H) {
        FirstStep<T> f;
        AmgLevelDev& L = H[0];
        f.dinv = Typed<T>::dinv(L);
        f.coef = Typed<T>::coef(L);
        f.x = as<T>(L.x0);
        f.d = as<T>(L.d);
        return f;
    }
    bool fuse_first(const std::vector<AmgLevelDev>& H) const { return H.size() > 1; }
    // y = (F + K) x
    // y = (F + K) x, scaled row-wise by rscale when given (the point-Jacobi
    // preconditioned operator diag(A)^{-1} A x in one pass)
    void applyA(const T* x, T* y, const FirstStep<T>* fs = nullptr, const T* rscale = nullptr) {
        RankOne<T> r = rank_one();
        if (r.slot_of)
            outlet_dot<T>(c->sym.n_out, c->d_optr, c->d_onode, Typed<T>::amsk(c), Typed<T>::ck(c), x, as<T>(c->d_s),
                          K.st);
        const double s = sizeof(T);
        const double bytes = (double)nnzb * (9 * s + col_bytes(c)) + 4.0 * (N + 1) + (rscale ? 9 : 6) * s * N;
        timed(c, NS_KT_SPMV_A, bytes, K.st, [&] {
            spmv<T>(3, 3, op(0, 0), x, y, T(1), nullptr, T(0), rscale, r.slot_of ? &r : nullptr, K.st, fs);
        });
    }
    // One V-cycle on level l for right-hand side b, result in xout.  On levels
    // l > 0 the caller has already done the first pre-smoothing step
    // (x = d = dinv b / theta into L.x0, L.d) inside the restriction kernel.
    void vcycle(std::vector<AmgLevelDev>& H, int l, const T* b, T* xout, bool first_done = false) {
        AmgLevelDev& L = H[l];
        const int bs = L.bs;
        const int64_t nv = (int64_t)L.n * bs;
        hipStream_t st = K.st;
        if (l + 1 == (int)H.size()) {
            dense_gemv<T>((int)nv, L.inv, b, xout, st);
            return;
        }
        const int degA = dflt(K.o.cheb_degree, kDefaultChebDegree);
        const int deg = &H == &sy.S ? dflt(K.o.cheb_degree_S, degA) : degA;
        const BlockOp<T> M = level_op(L);
        const T* dinv = Typed<T>::dinv(L);
        const T* coef = Typed<T>::coef(L);
        T* a = as<T>(L.x0);  // 2*deg-1 ping-pong flips: start in the scratch buffer, end in xout
        T* bb = xout;
        T* d = as<T>(L.d);
        const bool tme = (l == 0 && bs == 3);
        // finest S_hat level: applied in factored form D - C diag(A)^{-1} B
        const bool sfact = (l == 0 && &H == &sy.S);
        const double sz = sizeof(T);
        // algorithmic bytes: matrix values, columns and row pointers once; reads
        // x, b, dinv, the extra diagonal and d (steps after the first); writes d and x
        auto cheb = [&](const T* xi, T* xo, int step, const int32_t* agg, const T* ec) {
            const double cb = l == 0 ? col_bytes(c) : 4.0;
            const double bytes = (double)L.nnz * (9 * sz + cb) + 4.0 * (L.n + 1) + sz * nv * (step != 0 ? 7 : 6);
            if (tme)
                timed(c, NS_KT_CHEB_A0, bytes, st,
                      [&] { cheb_step<T>(bs, M, xi, xo, d, b, dinv, coef, step, agg, ec, st); });
            else if (sfact)
                this->sfact(xi, agg, ec, xo, T(1), nullptr, T(0), b, dinv, coef, step, d);
            else if (l == 1 && &H == &sy.S)
                timed(c, NS_KT_CHEB_S1, (double)L.nnz * (sz + 4) + 4.0 * (L.n + 1) + sz * nv * (step != 0 ? 7 : 6),
                      st, [&] { cheb_step<T>(bs, M, xi, xo, d, b, dinv, coef, step, agg, ec, st); });
            else
                cheb_step<T>(bs, M, xi, xo, d, b, dinv, coef, step, agg, ec, st);
        };
        // pre-smoothing from x = 0
        if (l == 0 && !first_done) cheb_first<T>(nv, b, dinv, coef, a, d, st);
        for (int s = 1; s < deg; ++s) {
            cheb(a, bb, s, nullptr, nullptr);
            std::swap(a, bb);
        }
        // coarse-grid correction: residual, restriction (+ first coarse step),
        // the coarse cycle, then post-smoothing -- gamma times on the levels
        // below the finest (gamma = 1: V-cycle, 2: W-cycle)
        AmgLevelDev& C = H[l + 1];
        const bool child_coarsest = (l + 2 == (int)H.size());
        T* xc = child_coarsest ? nullptr : as<T>(C.x0);
        const T* coefc = child_coarsest ? nullptr : Typed<T>::coef(C);
        const int gamma = l == 0 ? 1 : dflt(&H == &sy.S ? K.o.cycle_index_S : K.o.cycle_index_A, 1);
        for (int g = 0; g < gamma; ++g) {
        if (l == 0) {
            // finest level: a row-ordered residual SpMV (coalesced value
            // streams), then the restriction
            if (tme) {
                // same SpMV class as the A operator, plus reads of b and the extra diagonal
                const double bytes = (double)L.nnz * (9 * sz + col_bytes(c)) + 4.0 * (L.n + 1) + sz * nv * 4;
                timed(c, NS_KT_SPMV_A, bytes, st,
                      [&] { spmv<T>(bs, bs, M, a, as<T>(L.r), T(-1), b, T(1), nullptr, nullptr, st); });
            } else if (sfact) {
                this->sfact(a, nullptr, nullptr, as<T>(L.r), T(-1), b, T(1), nullptr, nullptr, nullptr, 0, nullptr);
            } else {
                spmv<T>(bs, bs, M, a, as<T>(L.r), T(-1), b, T(1), nullptr, nullptr, st);
            }
            restrict_first<T>(C.n, bs, L.aptr, L.anodes, as<T>(L.r), as<T>(C.b), xc, as<T>(C.d), Typed<T>::dinv(C),
                              coefc, coef + kCoefScale, st);
        } else {
            resid_restrict<T>(bs, M, a, b, C.n, L.aptr, L.anodes, as<T>(C.b), xc, as<T>(C.d), Typed<T>::dinv(C),
                              coefc, coef + kCoefScale, st);
        }
        vcycle(H, l + 1, as<T>(C.b), as<T>(C.x1));
        // post-smoothing; the first step applies the prolongated correction.
        // On a large finest A level, where the step streams from HBM, the
        // correction is added by a pass of its own instead: the fused step's
        // per-block aggregate gather costs more than that pass there (the
        // same addition either way).
        const bool pass = c->prolong_mode >= 0 ? c->prolong_mode == 1 : L.n >= kProlongPassRows;
        if (tme && pass) {
            prolong_add<T>(L.n, bs, L.agg, as<T>(C.x1), a, st);
            cheb(a, bb, 0, nullptr, nullptr);
        } else {
            cheb(a, bb, 0, L.agg, as<T>(C.x1));
        }
        std::swap(a, bb);
        for (int s = 1; s < deg; ++s) {
            cheb(a, bb, s, nullptr, nullptr);
            std::swap(a, bb);
        }
        }
        // (deg - 1) + gamma * deg buffer flips: an even count leaves the result
        // in the scratch buffer
        if (a != xout) axpby<T>(nv, T(1), a, T(0), nullptr, xout, st);
    }
    // P of an A-solve: pc_A for the intermediate ones, pc_I (if set) for the
    // inner ones of Algorithm 2
    int pc_of(bool inner) const { return inner && K.o.pc_I != 0 ? K.o.pc_I - 1 : K.o.pc_A; }
    void applyPA(const T* r, T* z, int pc) {
        if (pc == NS_PC_JACOBI)
            mul<T>(3 * (int64_t)N, Typed<T>::dinv(sy.A[0]), r, z, K.st);
        else
            vcycle(sy.A, 0, r, z);
    }
    // P_S: cycles_S steps of the stationary V-cycle iteration on S_hat from
    // zero, z <- z + V(r - S_hat z) (S_hat applied in factored form)
    void applyPS(const T* r, T* z, bool first_done = false) {
        vcycle(sy.S, 0, r, z, first_done);
        const int k = dflt(K.o.cycles_S, kDefaultCyclesS);
        T* t = as<T>(c->t_ps);
        T* e = t + N;
        for (int i = 1; i < k; ++i) {
            sfact(z, nullptr, nullptr, t, T(-1), r, T(1), nullptr, nullptr, nullptr, 0, nullptr);
            vcycle(sy.S, 0, t, e);
            axpby<T>(N, T(1), e, T(1), z, z, K.st);
        }
    }

    int solveA(const T* b, T* x, double rtol, bool inner = false) {
        const int pc = pc_of(inner);
        // inner solves with a P of their own use graphs of their own
        const int kind = pc == K.o.pc_A ? kKindA : kKindInner;
        std::function<void(const T*, T*)> sM, sP;
        bool fused = false;
        if (pc == NS_PC_JACOBI) {
            // point Jacobi applied in the operator's epilogue (the same product
            // diag(A)^{-1} (A v) as the separate scaling, one pass fewer)
            sM = [this](const T* in, T* out) { applyA(in, out, nullptr, Typed<T>::dinv(sy.A[0])); };
            fused = true;
        } else if (fuse_first(sy.A)) {
            sM = [this](const T* in, T* out) {
                const FirstStep<T> f = first_step(sy.A);
                applyA(in, out, &f);
            };
            sP = [this](const T* in, T* out) { vcycle(sy.A, 0, in, out, true); };
        }
        return gmres_left<T>(
            K, c->kw_A, 3 * (int64_t)N, [this](const T* in, T* out) { applyA(in, out); },
            [this, pc](const T* in, T* out) { applyPA(in, out, pc); }, b, x, rtol, dflt(K.o.m_A, 200),
            dflt(K.o.nmax_A, 200), kind, true, sM, sP, fused);
    }
    // Algorithm 2: y = D x - C A^{-1} (B x)
    void schur(const T* xp, T* y, const FirstStep<T>* fs = nullptr) {
        hipStream_t st = K.st;
        spmv<T>(1, 1, op(3, 3), xp, as<T>(c->t_xhat), T(1), nullptr, T(0), nullptr, nullptr, st);
        spmv<T>(3, 1, op(0, 3), xp, as<T>(c->t_xbar), T(1), nullptr, T(0), nullptr, nullptr, st);
        const int it = solveA(as<T>(c->t_xbar), as<T>(c->t_xt), dfltd(K.o.rtol_I, 1e-3), true);
        K.stats.inner_solves++;
        K.stats.inner_iters += it;
        spmv<T>(1, 3, op(3, 0), as<T>(c->t_xt), y, T(-1), as<T>(c->t_xhat), T(1), nullptr, nullptr, st, fs);
    }
    int solveS(const T* b, T* x) {
        std::function<void(const T*, T*)> sM, sP;
        if (fuse_first(sy.S)) {
            sM = [this](const T* in, T* out) {
                const FirstStep<T> f = first_step(sy.S);
                schur(in, out, &f);
            };
            sP = [this](const T* in, T* out) { applyPS(in, out, true); };
        }
        return gmres_left<T>(
            K, c->kw_S, N, [this](const T* in, T* out) { schur(in, out); },
            [this](const T* in, T* out) { applyPS(in, out); }, b, x, dfltd(K.o.rtol_S, 1e-3), dflt(K.o.m_S, 200),
            dflt(K.o.nmax_S, 200), kKindS, false, sM, sP);
    }
    // GMRES(m_S) on the sparse S_hat = D - C diag(A)^{-1} B, left
    // preconditioned by P_S (the Schur solve of SIMPLE); S_hat is applied in
    // factored form, so the operator launches kernels only and each Arnoldi
    // step is one graph.
    int solveShat(const T* b, T* x) {
        auto applyM = [this](const T* in, T* out) {
            sfact(in, nullptr, nullptr, out, T(1), nullptr, T(0), nullptr, nullptr, nullptr, 0, nullptr);
        };
        return gmres_left<T>(K, c->kw_S, N, applyM, [this](const T* in, T* out) { applyPS(in, out); }, b, x,
                             dfltd(K.o.rtol_S, 1e-3), dflt(K.o.m_S, 200), dflt(K.o.nmax_S, 200), kKindShat, true);
    }
    // SIMPLE (Sec. 3.2): y = P_SIMPLE^{-1} s, the factors of
    // [I 0; C A^{-1} I][A 0; 0 S_hat][I diag(A)^{-1} B; 0 I] inverted in turn.
    void simple(const T* s, T* y) {
        hipStream_t st = K.st;
        const int64_t n3 = 3 * (int64_t)N;
        const T* sv = s;
        const T* sp = s + n3;
        T* yhat = as<T>(c->t_yhat);
        int it = solveA(sv, yhat, dfltd(K.o.rtol_A, 1e-3));
        K.stats.a_solves++;
        K.stats.a_iters += it;
        spmv<T>(1, 3, op(3, 0), yhat, as<T>(c->t_tp), T(-1), sp, T(1), nullptr, nullptr, st);
        T* yp = y + n3;
        it = solveShat(as<T>(c->t_tp), yp);
        K.stats.s_solves++;
        K.stats.s_iters += it;
        T* tv = as<T>(c->t_tv);
        spmv<T>(3, 1, op(0, 3), yp, tv, T(1), nullptr, T(0), nullptr, nullptr, st);
        mul<T>(n3, Typed<T>::dinvA(sy), tv, tv, st);
        axpby<T>(n3, T(1), yhat, T(-1), tv, y, st);
    }
    void apply_pc(const T* s, T* y) {
        if (K.o.pc == NS_OUTER_SIMPLE)
            simple(s, y);
        else
            scr(s, y);
    }
    // Algorithm 3: y = P_SCR^{-1} s   (s, y: [4N], field-split)
    void scr(const T* s, T* y) {
        hipStream_t st = K.st;
        const T* sv = s;
        const T* sp = s + 3 * (int64_t)N;
        T* yhat = as<T>(c->t_yhat);
        int it = solveA(sv, yhat, dfltd(K.o.rtol_A, 1e-3));
        K.stats.a_solves++;
        K.stats.a_iters += it;
        spmv<T>(1, 3, op(3, 0), yhat, as<T>(c->t_tp), T(-1), sp, T(1), nullptr, nullptr, st);
        T* yp = y + 3 * (int64_t)N;
        it = solveS(as<T>(c->t_tp), yp);
        K.stats.s_solves++;
        K.stats.s_iters += it;
        spmv<T>(3, 1, op(0, 3), yp, as<T>(c->t_tv), T(-1), sv, T(1), nullptr, nullptr, st);
        it = solveA(as<T>(c->t_tv), y, dfltd(K.o.rtol_A, 1e-3));
        K.stats.a_solves++;
        K.stats.a_iters += it;
    }
};

// Outer FGMRES(m), right preconditioned, FP64 (Sec. 3).
template <typename T>
ns_status fgmres(Ctl& K, const double* b, double* x) {
    ns_ctx* c = K.c;
    hipStream_t st = K.st;
    KrylovWs& kw = c->kw_out;
    const int N = c->sym.N;
    const int64_t n = 4 * (int64_t)N;
    const int m = dflt(K.o.m, 200), nmax = dflt(K.o.nmax, 200);
    Nested<T> P(K);
    Nested<double> P64(K);
    RankOne<double> r1 = P64.rank_one();
    auto applyFull = [&](const double* in, double* out, double alpha, const double* z, double beta) {
        if (r1.slot_of)
            outlet_dot<double>(c->sym.n_out, c->d_optr, c->d_onode, c->d_a_msk, c->d_ck, in, c->d_s, st);
        const double bytes = (double)c->sym.g.nnz() * (16 * 8 + 4) + 4.0 * (N + 1) + 8.0 * 8 * N + (z ? 32.0 * N : 0);
        timed(c, NS_KT_SPMV_FULL, bytes, st, [&] {
            spmv_full<double>(N, c->d_rp, c->d_col, K.sy->V64, c->sym.g.nnz(), in, out, alpha, z, beta,
                              r1.slot_of ? &r1 : nullptr, st);
        });
    };
    int forced;
    const int idx = K.sc.begin(forced);
    double* V = kw.V;
    double* Z = kw.Z;
    const double bnorm = dev_norm<double>(c, n, b, kw.status + 4, st);
    if (bnorm == 0.0 || forced == 0) {
        fill<double>(n, 0.0, x, st);
        K.sc.end(idx, 0);
        K.stats.true_rel_res = 0.0;
        HIPCHK(hipStreamSynchronize(st));
        return NS_OK;
    }
    const double tol = std::max(dfltd(K.o.rtol, 1e-8) * bnorm, K.o.atol);
    fill<double>(n, 0.0, x, st);
    convert<double, double>(n, b, V, st);  // V_0 = b / ||b|| (the norm is already in status[4])
    double beta = bnorm;
    int total = 0;
    while (true) {
        scale_by<double>(n, V, kw.status + 4, true, V, st);
        init_g(kw.g, m + 1, beta, st);
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double* vj = V + (int64_t)j * kw.ld;
            double* zj = Z + (int64_t)j * kw.ld;
            if (std::is_same<T, double>::value) {
                P.apply_pc(reinterpret_cast<const T*>(vj), reinterpret_cast<T*>(zj));
            } else {
                convert<double, T>(n, vj, as<T>(c->t_s), st);
                P.apply_pc(as<T>(c->t_s), as<T>(c->t_yp));
                convert<T, double>(n, as<T>(c->t_yp), zj, st);
            }
            run_step(c, K, kKindOuter, j, [&] {
                applyFull(zj, V + (int64_t)(j + 1) * kw.ld, 1.0, nullptr, 0.0);
                cgs2_launch<double>(c, kw, n, j, V, st);
            });
            double resid;
            bool bd;
            read_step_status(c, kw, st, resid, bd);
            ++total;
            k = j + 1;
            const bool done = forced >= 0 ? total >= forced : resid <= tol;
            if (done || bd || total >= nmax) break;
        }
        backsolve(k, kw.m + 1, kw.H, kw.g, kw.y, st);  // H is stored with the workspace leading dimension
        combine<double, double>(n, k, Z, kw.ld, kw.y, x, true, st);
        // true residual in FP64
        applyFull(x, V, -1.0, b, 1.0);
        check_launch();
        beta = dev_norm<double>(c, n, V, kw.status + 4, st);
        if (!std::isfinite(beta)) throw Fail{NS_ERR_NAN, "true residual is not finite"};
        if (forced >= 0) {
            if (total >= forced || beta == 0.0) break;
        } else if (beta <= tol || total >= nmax || beta == 0.0) {
            break;
        }
    }
    K.sc.end(idx, total);
    K.stats.outer_iters = total;
    K.stats.true_rel_res = beta / bnorm;
    return beta <= tol || forced >= 0 ? NS_OK : NS_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// per-step set-up: diag(A) with the lumped rank-one diagonal, S_hat, AMG
// numeric (Galerkin sums, Jacobi diagonals, lambda_max, coarsest inverse)
// ---------------------------------------------------------------------------

// Upper end of the smoother interval of a level: the smaller of the
// Gershgorin bound of D^{-1} M (guaranteed) and kPowerSafety times the
// estimate from kPowerIters power iterations (which approach the spectral
// radius from below) from the fixed start vector.  The iterates are not
// normalised (the estimate ||y_k|| / ||y_{k-1}|| equals the normalised
// iteration's last norm; the growth lambda^k stays far inside FP64 range).
// Writes ||y_k||, ||y_{k-1}|| and the Gershgorin bound to out[0..2].
constexpr int kPowerIters = 20;
constexpr double kPowerSafety = 1.2;
// red: reduction partials of this chain (at least n/1024 + 1 doubles), so
// chains of different levels can run concurrently
void smoother_bound_dev(ns_ctx* c, const BlockOp<double>& M, int bs, const double* dinv, double* x, double* y,
                        double* red, double* out, hipStream_t st) {
    const int64_t n = (int64_t)M.n * bs;
    power_start(n, x, st);
    for (int it = 0; it < kPowerIters; ++it) {
        spmv<double>(bs, bs, M, x, y, 1.0, nullptr, 0.0, dinv, nullptr, st);
        std::swap(x, y);
    }
    norm2<double>(n, x, out, red, st);
    norm2<double>(n, y, out + 1, red, st);
    // the iterates are no longer needed: x holds the per-block partials
    // (at most n/4 + 1 <= n*bs of them)
    gershgorin_bound(M, bs, dinv, x, out + 2, st);
    check_launch();
}
double smoother_bound_host(const double* v) { return std::min(v[2], kPowerSafety * (v[0] / v[1])); }

// Numeric per-step set-up on the device: diag(A) with the lumped rank-one
// diagonal, then independent chains on four streams -- S_hat, its Galerkin
// levels and coarsest inverse on `st`; the A hierarchy's Galerkin levels and
// coarsest inverse on aux[0]; the smoother-bound power iterations of the A
// levels on aux[1], of the finest S_hat level on aux[2] (as soon as S_hat
// exists) and of the coarser S_hat levels on aux[3].  Every chain works in
// buffers of its own level (the power iterations: the level's x0, r and b as
// iterates and reduction partials); all streams rejoin `st` at the end.
void setup_device(ns_ctx* c, SystemDev& y, hipStream_t st) {
    const Symbolic& S = c->sym;
    const int N = S.N;
    const int64_t nnzb = S.g.nnz();
    const int L = (int)S.lv.size();
    fill<double>(3 * (int64_t)N, 0.0, y.dK64, st);
    rank_one_diag((int)S.onode.size(), c->d_onode, c->d_oid, c->d_a_msk, c->d_ck, y.dK64, st);
    block_dinv(N, 3, c->d_rp, c->d_col, y.V64, 4 * nnzb, nnzb, y.dK64, y.dinvA64, y.diagA64, st);
    double* bnd = c->d_bnd;
    hipStream_t sA = c->aux[0], sAp = c->aux[1], sSp = c->aux[2], sSc = c->aux[3];
    HIPCHK(hipEventRecord(c->fork_ev, st));
    HIPCHK(hipStreamWaitEvent(sA, c->fork_ev, 0));
    auto bounds = [&](int h, int l0, int l1, hipStream_t ps) {  // levels l0 <= l < l1, smoothed ones only
        std::vector<AmgLevelDev>& H = h == 0 ? y.A : y.S;
        for (int l = l0; l < l1 && l + 1 < L; ++l) {
            AmgLevelDev& d = H[l];
            BlockOp<double> M;
            M.n = d.n;
            M.rp = d.rp;
            M.col = d.col;
            if (d.col == c->d_col) M.dcol = dcol_of(c);
            M.v = d.v64;
            M.rs = d.rstride;
            M.cs = d.cstride;
            M.dextra = d.dextra64;
            M.lanes = lanes_for(d.nnz, d.n, d.bs);
            M.unroll = unroll_of(c, d.nnz, d.n);
            smoother_bound_dev(c, M, d.bs, d.dinv64, d.x0, d.r, d.b, bnd + 3 * (h * L + l), ps);
        }
    };
    auto coarsest = [&](std::vector<AmgLevelDev>& H, hipStream_t cs) {
        AmgLevelDev& d = H[L - 1];
        dense_from_csr(d.n, d.bs, d.rp, d.col, d.v64, d.rstride, d.cstride, d.dextra64, d.work, cs);
        gauss_jordan_inverse2(d.n * d.bs, d.work, d.inv, 0, nullptr, nullptr, cs);
    };
    // The chains are queued in the order in which they can start on the
    // device: S_hat and the finest S_hat diagonal, the A Galerkin levels, then
    // the finest S_hat level's power iterations (the longest chain), the A
    // coarsest inverse, the A power iterations, and last the S_hat Galerkin
    // levels with their power iterations and coarsest inverse.  A chain with
    // no kernels (hierarchies of one or two levels) is skipped.
    const int sys = &y == &c->sys[0] ? 0 : 1;
    auto chain = [&](int id, bool nonempty, hipStream_t cs, auto&& body) {
        if (nonempty) run_chain(c, sys, id, cs, body);
    };
    shat_numeric(N, c->d_rp, c->d_col, y.V64, nnzb, y.dinvA64, c->d_srp, c->d_scol, y.shat64, st);
    block_dinv(N, 1, c->d_srp, c->d_scol, y.shat64, 0, 0, nullptr, y.S[0].dinv64, nullptr, st);
    HIPCHK(hipEventRecord(c->aux_ev[3], st));
    HIPCHK(hipStreamWaitEvent(sSp, c->aux_ev[3], 0));
    chain(0, L > 1, sA, [&] {
        for (int l = 1; l < L; ++l) {
            AmgLevelDev& f = y.A[l - 1];
            AmgLevelDev& a = y.A[l];
            galerkin(a.nnz, 3, 3, a.gptr, a.gidx, f.v64, f.rstride, f.cstride, a.v64, a.rstride, a.cstride,
                     a.qrow, a.col, l == 1 ? y.dK64 : nullptr, f.aptr, f.anodes, sA);
            block_dinv(a.n, 3, a.rp, a.col, a.v64, a.rstride, a.cstride, nullptr, a.dinv64, nullptr, sA);
        }
        check_launch();
    });
    HIPCHK(hipEventRecord(c->aux_ev[0], sA));
    chain(1, L > 1, sSp, [&] { bounds(1, 0, 1, sSp); });
    chain(2, true, sA, [&] {
        coarsest(y.A, sA);
        check_launch();
    });
    HIPCHK(hipStreamWaitEvent(sAp, c->aux_ev[0], 0));
    chain(3, L > 1, sAp, [&] { bounds(0, 0, L, sAp); });
    chain(4, L > 1, st, [&] {
        for (int l = 1; l < L; ++l) {
            AmgLevelDev& fs = y.S[l - 1];
            AmgLevelDev& s = y.S[l];
            galerkin(s.nnz, 1, 1, s.gptr, s.gidx, fs.v64, 0, 0, s.v64, 0, 0, nullptr, s.col, nullptr, nullptr,
                     nullptr, st);
            block_dinv(s.n, 1, s.rp, s.col, s.v64, 0, 0, nullptr, s.dinv64, nullptr, st);
        }
        check_launch();
    });
    HIPCHK(hipEventRecord(c->aux_ev[1], st));
    HIPCHK(hipStreamWaitEvent(sSc, c->aux_ev[1], 0));
    chain(5, L > 2, sSc, [&] { bounds(1, 1, L, sSc); });
    chain(6, true, st, [&] {
        coarsest(y.S, st);
        check_launch();
    });
    check_launch();
    const hipStream_t joins[4] = {sA, sAp, sSp, sSc};
    for (int k = 0; k < 4; ++k) {
        HIPCHK(hipEventRecord(c->aux_ev[k], joins[k]));
        HIPCHK(hipStreamWaitEvent(st, c->aux_ev[k], 0));
    }
}

void convert32(ns_ctx* c, SystemDev& y, hipStream_t st);

void setup_system(ns_ctx* c, SystemDev& y, bool need32, hipStream_t st) {
    const Symbolic& S = c->sym;
    const int N = S.N;
    const int64_t nnzb = S.g.nnz();
    const int L = (int)S.lv.size();
    if (!y.ready || y.version != c->version) {
        // (one graph spanning all four streams replayed 1.4 ms slower than
        // direct launches; a graph per stream's chain keeps the streams' overlap)
        setup_device(c, y, st);
        double* bnd = c->d_bnd;
        std::vector<double> hb(3 * 2 * (size_t)L);
        HIPCHK(hipMemcpyAsync(hb.data(), bnd, hb.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int h = 0; h < 2; ++h)
            for (int l = 0; l + 1 < L; ++l) {
                AmgLevelDev& d = h == 0 ? y.A[l] : y.S[l];
                d.lmax = smoother_bound_host(&hb[3 * (h * L + l)]);
                if (!std::isfinite(d.lmax) || !(d.lmax > 0.0))
                    throw Fail{NS_ERR_NAN, "AMG smoother bound is not finite and positive"};
            }
        y.ready = true;
        y.have32 = false;
        y.coef_deg = 0;
        y.version = c->version;
    }
    if (need32 && !y.have32) {
        run_chain(c, &y == &c->sys[0] ? 0 : 1, 7, st, [&] { convert32(c, y, st); });
        y.have32 = true;
    }
}

// FP32 copies of the tangent planes, diagonals, S_hat, the AMG levels and
// the rank-one data, for the FP32-inner solves
void convert32(ns_ctx* c, SystemDev& y, hipStream_t st) {
    const Symbolic& S = c->sym;
    const int N = S.N;
    const int64_t nnzb = S.g.nnz();
    const int L = (int)S.lv.size();
    if (c->ell32)
        to_ell<double, float>(N, S.ell, c->d_rp, y.V64, nnzb, 16, y.V32, st);
    else
        convert<double, float>(nnzb * 16, y.V64, y.V32, st);
    convert<double, float>(3 * (int64_t)N, y.dK64, y.dK32, st);
    convert<double, float>(3 * (int64_t)N, y.dinvA64, y.dinvA32, st);
    convert<double, float>(S.shat.nnz(), y.shat64, y.shat32, st);
    for (int h = 0; h < 2; ++h) {
        std::vector<AmgLevelDev>& H = h == 0 ? y.A : y.S;
        for (int l = 0; l < L; ++l) {
            AmgLevelDev& d = H[l];
            if (l > 0) convert<double, float>(d.nnz * d.bs * d.bs, d.v64, d.v32, st);
            if (!(h == 0 && l == 0)) convert<double, float>((int64_t)d.n * d.bs, d.dinv64, d.dinv32, st);
        }
    }
    const int nslot = (int)S.onode.size();
    convert<double, float>(3 * (int64_t)nslot, c->d_a_msk, c->d_a_msk32, st);
    convert<double, float>(S.n_out, c->d_ck, c->d_ck32, st);
    check_launch();
}

// Chebyshev coefficients of every smoothed level: interval
// [lmax/ratio, lmax] of D^{-1} M, theta/delta its centre/half-width.
// Step coefficients of the Chebyshev recurrence for every step up to the
// largest degree (a step's coefficients do not depend on the degree in use,
// so both hierarchies can run different degrees from one table).
void upload_coef(ns_ctx* c, SystemDev& y, int deg, double ratio, const double scale[2], hipStream_t st) {
    if (deg < 1 || deg > kMaxChebDegree) throw Fail{NS_ERR_ARG, "Chebyshev degree out of range [1, 8]"};
    if (!(ratio > 1.0) || !std::isfinite(ratio)) throw Fail{NS_ERR_ARG, "cheb_ratio must be finite and > 1"};
    deg = kMaxChebDegree;
    if (y.coef_deg == deg && y.coef_ratio == ratio && y.coef_scale[0] == scale[0] && y.coef_scale[1] == scale[1])
        return;
    std::vector<double> host;
    std::vector<AmgLevelDev*> lv;
    for (int h = 0; h < 2; ++h) {
        std::vector<AmgLevelDev>& H = h == 0 ? y.A : y.S;
        for (int l = 0; l + 1 < (int)H.size(); ++l) {
            const double lmax = H[l].lmax, lmin = lmax / ratio;
            const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
            std::vector<double> cf(kCoefLen, 0.0);
            cf[0] = 1.0 / theta;
            double rho = 1.0 / sigma;
            for (int s = 1; s < deg; ++s) {
                const double rn = 1.0 / (2.0 * sigma - rho);
                cf[2 * s - 1] = rn * rho;
                cf[2 * s] = 2.0 * rn / delta;
                rho = rn;
            }
            cf[kCoefScale] = scale[h];
            host.insert(host.end(), cf.begin(), cf.end());
            lv.push_back(&H[l]);
        }
    }
    for (size_t i = 0; i < lv.size(); ++i) {
        HIPCHK(hipMemcpyAsync(lv[i]->coef64, host.data() + i * kCoefLen, kCoefLen * sizeof(double),
                              hipMemcpyHostToDevice, st));
        convert<double, float>(kCoefLen, lv[i]->coef64, lv[i]->coef32, st);
    }
    check_launch();
    HIPCHK(hipStreamSynchronize(st));  // the host buffer goes out of scope
    y.coef_deg = deg;
    y.coef_ratio = ratio;
    y.coef_scale[0] = scale[0];
    y.coef_scale[1] = scale[1];
}

void upload_coef(ns_ctx* c, SystemDev& y, const ns_solve_opts& o, hipStream_t st) {
    const double scale[2] = {dfltd(o.cc_scale_A, kDefaultCcScaleA), dfltd(o.cc_scale_S, kDefaultCcScaleS)};
    upload_coef(c, y, dflt(o.cheb_degree, kDefaultChebDegree), dfltd(o.cheb_ratio, kDefaultChebRatio), scale, st);
}

void ensure_transposed(ns_ctx* c, hipStream_t st) {
    SystemDev& t = c->sys[1];
    if (t.ready && t.version == c->version) return;
    transpose_values(c->sym.g.nnz(), c->d_tmap, c->sys[0].V64, t.V64, st);
    check_launch();
    t.ready = false;
}

void check_solve_opts(const ns_solve_opts& o) {
    if (o.precision != NS_FP64 && o.precision != NS_FP32_INNER) throw Fail{NS_ERR_ARG, "unknown precision"};
    if (o.pc != NS_OUTER_SCR && o.pc != NS_OUTER_SIMPLE) throw Fail{NS_ERR_ARG, "unknown outer preconditioner"};
    if (o.pc_A != NS_PC_AMG && o.pc_A != NS_PC_JACOBI) throw Fail{NS_ERR_ARG, "unknown P_A"};
    if (o.pc_I < 0 || o.pc_I > 2) throw Fail{NS_ERR_ARG, "unknown P of the inner A-solves"};
    if (o.reserved != 0) throw Fail{NS_ERR_ARG, "reserved option field must be 0"};
    if (o.cheb_degree < 0 || o.cheb_degree > kMaxChebDegree || o.cheb_degree_S < 0 ||
        o.cheb_degree_S > kMaxChebDegree)
        throw Fail{NS_ERR_ARG, "Chebyshev degree out of range [1, 8]"};
    if (o.cycle_index_A < 0 || o.cycle_index_A > 3 || o.cycle_index_S < 0 || o.cycle_index_S > 3)
        throw Fail{NS_ERR_ARG, "AMG cycle index out of range [1, 3]"};
    for (double sc : {o.cc_scale_A, o.cc_scale_S})
        if (!(sc >= 0.0 && sc <= 2.0)) throw Fail{NS_ERR_ARG, "coarse-grid correction scale out of range [0, 2]"};
}

ns_status run_solve(ns_ctx* c, int which, const ns_solve_opts* opts, const double* b, double* x, ns_stats* hs,
                    hipStream_t st) {
    if (!c->bound) throw Fail{NS_ERR_STATE, "context not bound"};
    if (!c->assembled) throw Fail{NS_ERR_STATE, "no tangent assembled"};
    if (!b || !x) throw Fail{NS_ERR_ARG, "null vector"};
    Ctl K{};
    K.c = c;
    K.st = st;
    if (opts) K.o = *opts;
    K.o.atol = K.o.atol > 0 ? K.o.atol : 1e-50;
    if (dflt(K.o.m, 200) > c->kw_out.m || dflt(K.o.m_A, 200) > c->kw_A.m || dflt(K.o.m_S, 200) > c->kw_S.m)
        throw Fail{NS_ERR_ARG, "restart length exceeds the context's Krylov workspace"};
    check_solve_opts(K.o);
    K.sc.replay = K.o.h_sched;
    K.sc.replay_len = K.o.sched_len;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(st));  // inputs produced on the caller's stream
    st = c->own;
    K.st = st;
    auto t0 = std::chrono::steady_clock::now();
    if (which == 1) ensure_transposed(c, st);
    K.sy = &c->sys[which];
    setup_system(c, *K.sy, K.o.precision == NS_FP32_INNER, st);
    upload_coef(c, *K.sy, K.o, st);
    HIPCHK(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    ns_status rs = K.o.precision == NS_FP32_INNER ? fgmres<float>(K, b, x) : fgmres<double>(K, b, x);
    HIPCHK(hipStreamSynchronize(st));
    auto t2 = std::chrono::steady_clock::now();
    timing_collect(c);
    K.stats.setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    K.stats.solve_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
    K.stats.n_calls = (int)K.sc.log.size();
    K.stats.amg_levels_A = K.stats.amg_levels_S = (int)c->sym.lv.size();
    if (K.o.h_sched_out)
        for (int i = 0; i < (int)K.sc.log.size() && i < K.o.sched_cap; ++i) K.o.h_sched_out[i] = K.sc.log[i];
    if (hs) *hs = K.stats;
    return rs;
}

template <typename F>
ns_status guard(ns_ctx* c, F&& f) {
    try {
        return f();
    } catch (const Fail& e) {
        if (c) c->err = e.msg;
        return e.st;
    } catch (const std::exception& e) {
        if (c) c->err = e.what();
        return NS_ERR_ARG;
    }
}

// Three-element Windkessel over one time step (Algorithm 1): n_ts steps of the
// Runge-Kutta scheme with K2, K3 at the thirds of each sub-interval and weights
// 1/8, 3/8, 3/8, 1/8, the flow rate interpolated linearly between Q_n and
// Q_np1.  Returns P_{n+1} = R_p Q_np1 + Pi_{n+1} + P_d and Pi_{n+1} in *Pi_end.
// C == 0: resistance model (R_p + R_d) Q + P_d, Pi_end = 0.
double windkessel(double Rp, double C, double Rd, double Pd, double Pi_n, double Q_n, double Q_np1, int nts,
                  double dt, double* Pi_end) {
    if (C == 0.0) {
        if (Pi_end) *Pi_end = 0.0;
        return (Rp + Rd) * Q_np1 + Pd;
    }
    const double h = dt / nts;
    auto F = [&](double Pi, double Q) { return -Pi / (Rd * C) + Q / C; };
    auto Qm = [&](int m) { return (1.0 - (double)m / nts) * Q_n + ((double)m / nts) * Q_np1; };
    double Pi = Pi_n;
    for (int m = 0; m < nts; ++m) {
        const double q0 = Qm(m), q1 = Qm(m + 1);
        const double k1 = F(Pi, q0);
        const double k2 = F(Pi + k1 * h / 3.0, 2.0 * q0 / 3.0 + q1 / 3.0);
        const double k3 = F(Pi - k1 * h / 3.0 + k2 * h, q0 / 3.0 + 2.0 * q1 / 3.0);
        const double k4 = F(Pi + k1 * h - k2 * h + k3 * h, q1);
        Pi = Pi + k1 * h / 8.0 + 3.0 * k2 * h / 8.0 + 3.0 * k3 * h / 8.0 + k4 * h / 8.0;
    }
    if (Pi_end) *Pi_end = Pi;
    return Rp * Q_np1 + Pi + Pd;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

ns_status ns_ctx_create(const ns_mesh* mesh, const ns_ctx_opts* opts, ns_ctx** out, size_t* workspace_bytes) {
    if (!mesh || !out || !workspace_bytes) {
        g_create_err = "null argument";
        return NS_ERR_ARG;
    }
    *out = nullptr;
    ns_ctx* c = new ns_ctx();
    if (opts) c->opts = *opts;
    try {
        std::string e = build_symbolic(mesh, c->opts, c->sym);
        if (!e.empty()) {
            g_create_err = e;
            delete c;
            return NS_ERR_ARG;
        }
        c->h_xyz.assign(mesh->h_xyz, mesh->h_xyz + 3 * (size_t)mesh->n_nodes);
        c->h_mask.assign(mesh->h_dirichlet, mesh->h_dirichlet + 4 * (size_t)mesh->n_nodes);
        Arena A;
        layout(c, A);
        c->ws_bytes = A.off + 256;
    } catch (const std::exception& ex) {
        g_create_err = ex.what();
        delete c;
        return NS_ERR_ARG;
    }
    *workspace_bytes = c->ws_bytes;
    *out = c;
    return NS_OK;
}

ns_status ns_ctx_bind(ns_ctx* c, void* ws, size_t bytes, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!ws || bytes < c->ws_bytes) throw Fail{NS_ERR_WORKSPACE, "workspace missing or too small"};
        if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) throw Fail{NS_ERR_WORKSPACE, "workspace not 256-byte aligned"};
        HIPCHK(hipGetDevice(&c->device));
        // a new workspace holds no tangent yet, and captured graphs hold
        // pointers into the previous one
        for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        c->graphs.clear();
        c->assembled = false;
        for (SystemDev& y : c->sys) {
            y.ready = false;
            y.have32 = false;
            y.coef_deg = 0;
        }
        Arena A;
        A.base = static_cast<char*>(ws);
        layout(c, A);
        const Symbolic& S = c->sym;
        h2d(c->d_rp, S.g.rp, st);
        h2d(c->d_col, S.g.col, st);
        if (c->d_dcol) h2d(c->d_dcol, S.dcol, st);
        if (c->d_dcol_ell) h2d(c->d_dcol_ell, S.dcol_ell, st);
        h2d(c->d_diag, S.diag_pos, st);
        h2d(c->d_rowof, S.row_of, st);
        h2d(c->d_tmap, S.tmap, st);
        h2d(c->d_tets, S.tets, st);
        h2d(c->d_emap, S.emap, st);
        h2d(c->d_faces, S.faces, st);
        h2d(c->d_fmap, S.fmap, st);
        h2d(c->d_fslot, S.fslot, st);
        h2d(c->d_face_out, S.face_out, st);
        h2d(c->d_onode, S.onode, st);
        h2d(c->d_oid, S.oid, st);
        h2d(c->d_slot_of, S.slot_of, st);
        h2d(c->d_optr, S.optr, st);
        h2d(c->d_srp, S.shat.rp, st);
        h2d(c->d_scol, S.shat.col, st);
        h2d(c->d_xyz, c->h_xyz, st);
        h2d(c->d_mask, c->h_mask, st);
        for (int l = 1; l < (int)S.lv.size(); ++l) {
            const AmgLevelSym& ls = S.lv[l];
            AmgLevelDev& a = c->sys[0].A[l];
            AmgLevelDev& s = c->sys[0].S[l];
            h2d(a.rp, ls.a.rp, st);
            h2d(a.col, ls.a.col, st);
            h2d(s.rp, ls.s.rp, st);
            h2d(s.col, ls.s.col, st);
            h2d(a.gptr, ls.gptr, st);
            h2d(a.gidx, ls.gidx, st);
            h2d(a.qrow, ls.a_qrow, st);
            h2d(s.gptr, ls.sgptr, st);
            h2d(s.gidx, ls.sgidx, st);
        }
        for (int l = 0; l + 1 < (int)S.lv.size(); ++l) {
            const AmgLevelSym& ls = S.lv[l];
            AmgLevelDev& a = c->sys[0].A[l];
            h2d(a.agg, ls.agg, st);
            h2d(a.aptr, ls.aptr, st);
            h2d(a.anodes, ls.anodes, st);
        }
        // outlet vectors a^k (geometry only)
        const int nslot = (int)S.onode.size();
        fill<double>(std::max(1, 3 * nslot), 0.0, c->d_a_raw, st);
        for (int fc = 0; fc < S.n_fcolors; ++fc)
            outlet_vectors(S.fcolor_ptr[fc], S.fcolor_ptr[fc + 1] - S.fcolor_ptr[fc], c->d_faces, c->d_fslot,
                           c->d_xyz, c->d_a_raw, st);
        mask_outlet(nslot, c->d_onode, c->d_mask, c->d_a_raw, c->d_a_msk, st);
        check_launch();
        if (!c->h_pinned) HIPCHK(hipHostMalloc((void**)&c->h_pinned, 64 * sizeof(double), hipHostMallocDefault));
        if (!c->h_mapped) {
            HIPCHK(hipHostMalloc((void**)&c->h_mapped, 64 * sizeof(double),
                                 hipHostMallocMapped | hipHostMallocCoherent));
            HIPCHK(hipHostGetDevicePointer((void**)&c->d_mapped, c->h_mapped, 0));
            std::memset(c->h_mapped, 0, 64 * sizeof(double));
        }
        c->step_seq = 0;
        c->slot_seq[0] = c->slot_seq[1] = 0;
        std::memset(c->h_mapped + kMapSeq, 0, 2 * sizeof(double));
        if (!c->own) HIPCHK(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
        // the scratch of ns_resistance_gradient_noalloc on this device
        HIPCHK(noalloc_scratch(c->device, &c->noalloc_scratch));
        for (int e = 0; e < 2; ++e)
            if (!c->step_ev[e]) HIPCHK(hipEventCreateWithFlags(&c->step_ev[e], hipEventDisableTiming));
        for (int a = 0; a < ns_ctx::kAux; ++a) {
            if (!c->aux[a]) HIPCHK(hipStreamCreateWithFlags(&c->aux[a], hipStreamNonBlocking));
            if (!c->aux_ev[a]) HIPCHK(hipEventCreateWithFlags(&c->aux_ev[a], hipEventDisableTiming));
        }
        if (!c->fork_ev) HIPCHK(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
        // Captured graphs pay off only where launches dominate: replayed, they
        // ran 10-20 % faster than direct launches on meshes of ~700 nodes but
        // 2-4 % slower from ~1600 nodes up (every measured mesh to 2e5 nodes).
        // NS_GRAPHS=0/1 forces the choice.
        const char* ng = getenv("NS_GRAPHS");
        c->use_graphs = (ng && (ng[0] == '0' || ng[0] == '1')) ? ng[0] == '1' : S.N <= kGraphMaxNodes;
        const char* xr = getenv("NS_XCD_ROWS");
        c->xcd_mode = (xr && (xr[0] == '0' || xr[0] == '1')) ? xr[0] - '0' : -1;
        const char* pp = getenv("NS_PROLONG_PASS");
        c->prolong_mode = (pp && (pp[0] == '0' || pp[0] == '1')) ? pp[0] - '0' : -1;
        const char* cs16 = getenv("NS_COL16");
        c->col16 = c->d_dcol != nullptr && !(cs16 && cs16[0] == '0');
        const char* ce = getenv("NS_ELL");
        c->ell32 = c->col16 && c->d_dcol_ell != nullptr && !(ce && ce[0] == '0');
        const char* ru = getenv("NS_ROW_UNROLL");
        c->unroll_mode = (ru && (ru[0] == '2' || ru[0] == '4') && ru[1] == '\0') ? ru[0] - '0' : -1;
        HIPCHK(hipStreamSynchronize(st));
        c->bound = true;
        return NS_OK;
    });
}

void ns_ctx_destroy(ns_ctx* c) {
    if (!c) return;
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->h_mapped) (void)hipHostFree(c->h_mapped);
    for (hipEvent_t e : c->kt_ev) (void)hipEventDestroy(e);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    for (int e = 0; e < 2; ++e)
        if (c->step_ev[e]) (void)hipEventDestroy(c->step_ev[e]);
    for (int a = 0; a < ns_ctx::kAux; ++a) {
        if (c->aux[a]) (void)hipStreamSynchronize(c->aux[a]);
        if (c->aux_ev[a]) (void)hipEventDestroy(c->aux_ev[a]);
        if (c->aux[a]) (void)hipStreamDestroy(c->aux[a]);
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->own) (void)hipStreamDestroy(c->own);
    delete c;
}

const char* ns_last_error(const ns_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

ns_status ns_outlet_flow(ns_ctx* c, const double* d_v, double* h_Q, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->bound) throw Fail{NS_ERR_STATE, "context not bound"};
        const int NO = c->sym.n_out;
        if (NO == 0) return NS_OK;
        if (!d_v || !h_Q) throw Fail{NS_ERR_ARG, "null argument"};
        outlet_dot<double>(NO, c->d_optr, c->d_onode, c->d_a_raw, nullptr, d_v, c->d_s, st);
        check_launch();
        HIPCHK(hipMemcpyAsync(h_Q, c->d_s, NO * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return NS_OK;
    });
}

ns_status ns_rank_one_dots(ns_ctx* c, const double* d_xv, double* h_out, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->bound) throw Fail{NS_ERR_STATE, "context not bound"};
        const int NO = c->sym.n_out;
        if (NO == 0) return NS_OK;
        if (!d_xv || !h_out) throw Fail{NS_ERR_ARG, "null argument"};
        outlet_dot<double>(NO, c->d_optr, c->d_onode, c->d_a_msk, nullptr, d_xv, c->d_s, st);
        check_launch();
        HIPCHK(hipMemcpyAsync(h_out, c->d_s, NO * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return NS_OK;
    });
}

ns_status ns_resistance_gradient(ns_ctx* c, const double* d_lambda, const double* d_x, double* h_grad,
                                 hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->bound) throw Fail{NS_ERR_STATE, "context not bound"};
        if (!c->assembled || !c->resistance_mode)
            throw Fail{NS_ERR_STATE, "the last assembly did not take resistance outlets"};
        const int NO = c->sym.n_out;
        if (NO == 0) return NS_OK;
        if (!d_lambda || !d_x || !h_grad) throw Fail{NS_ERR_ARG, "null argument"};
        HIPCHK(hipSetDevice(c->device));
        outlet_dot<double>(NO, c->d_optr, c->d_onode, c->d_a_msk, nullptr, d_lambda, c->d_s2, st);
        outlet_dot<double>(NO, c->d_optr, c->d_onode, c->d_a_msk, nullptr, d_x, c->d_grad, st);
        resistance_grad(NO, c->d_s2, c->d_grad, c->d_Q, c->a_f, c->c_f, c->d_grad, st);
        check_launch();
        HIPCHK(hipMemcpyAsync(h_grad, c->d_grad, NO * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return NS_OK;
    });
}

ns_status ns_gen_alpha(double rho_inf, double* h_out3) {
    if (!h_out3 || !(rho_inf >= 0.0 && rho_inf <= 1.0)) return NS_ERR_ARG;
    h_out3[0] = 0.5 * (3.0 - rho_inf) / (1.0 + rho_inf);
    h_out3[1] = 1.0 / (1.0 + rho_inf);
    h_out3[2] = h_out3[1];
    return NS_OK;
}

ns_status ns_assemble_tangent(ns_ctx* c, const ns_phys* ph, const double* d_v, const double* d_p,
                              const double* d_vdot, double* d_rhs, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->bound) throw Fail{NS_ERR_STATE, "context not bound"};
        if (!ph || !d_v || !d_p || !d_vdot || !d_rhs) throw Fail{NS_ERR_ARG, "null argument"};
        const Symbolic& S = c->sym;
        const bool resist = S.n_out > 0 && ph->h_R;
        if (S.n_out > 0 && !resist && (!ph->h_m || !ph->h_P_af)) throw Fail{NS_ERR_ARG, "outlet data missing"};
        if (!(ph->rho > 0) || !(ph->dt > 0) || ph->mu < 0 || ph->rho_inf < 0 || ph->rho_inf > 1)
            throw Fail{NS_ERR_ARG, "invalid physical parameters"};
        HIPCHK(hipSetDevice(c->device));
        const double am = 0.5 * (3.0 - ph->rho_inf) / (1.0 + ph->rho_inf);
        const double af = 1.0 / (1.0 + ph->rho_inf), gam = af;
        const double cf = af * gam * ph->dt;
        const double beta = ph->beta_bf > 0 ? ph->beta_bf : 0.2;
        const int64_t nnzb = S.g.nnz();
        fill<double>(nnzb * 16, 0.0, c->d_aos, st);
        fill<double>(4 * (int64_t)S.N, 0.0, c->d_res, st);
        AsmArgs a;
        a.tets = c->d_tets;
        a.emap = c->d_emap;
        a.xyz = c->d_xyz;
        a.v = d_v;
        a.p = d_p;
        a.vdot = d_vdot;
        a.aos = c->d_aos;
        a.res = c->d_res;
        a.N = S.N;
        a.rho = ph->rho;
        a.mu = ph->mu;
        a.dt = ph->dt;
        a.c_m = am;
        a.c_f = cf;
        a.c_t = ph->c_t > 0 ? ph->c_t : 4.0;
        a.c_i = ph->c_i > 0 ? ph->c_i : 36.0;
        for (int col = 0; col < S.n_colors; ++col) {
            a.E0 = S.color_ptr[col];
            a.count = S.color_ptr[col + 1] - S.color_ptr[col];
            assemble_elements(a, st);
        }
        if (S.n_out > 0) {
            const int NO = S.n_out;
            if (resist) {
                // resistance outlets: Q^k (given, or a^k . v on the device), then
                // c_k and P^k_{n+af} on the device
                c->h_outlets.assign(ph->h_R, ph->h_R + NO);
                if (ph->h_P_n) c->h_outlets.insert(c->h_outlets.end(), ph->h_P_n, ph->h_P_n + NO);
                if (ph->h_Q) c->h_outlets.insert(c->h_outlets.end(), ph->h_Q, ph->h_Q + NO);
                HIPCHK(hipMemcpyAsync(c->d_R, c->h_outlets.data(), NO * sizeof(double), hipMemcpyHostToDevice, st));
                size_t off = NO;
                if (ph->h_P_n) {
                    HIPCHK(hipMemcpyAsync(c->d_Pn, c->h_outlets.data() + off, NO * sizeof(double),
                                          hipMemcpyHostToDevice, st));
                    off += NO;
                }
                if (ph->h_Q)
                    HIPCHK(hipMemcpyAsync(c->d_Q, c->h_outlets.data() + off, NO * sizeof(double),
                                          hipMemcpyHostToDevice, st));
                else
                    outlet_dot<double>(NO, c->d_optr, c->d_onode, c->d_a_raw, nullptr, d_v, c->d_Q, st);
                resistance_outlets(NO, c->d_R, ph->h_P_n ? c->d_Pn : nullptr, c->d_Q, af, cf, c->d_ck, c->d_Paf, st);
            } else {
                std::vector<double> paf(ph->h_P_af, ph->h_P_af + NO);
                c->ck_host.resize(NO);
                for (int k = 0; k < NO; ++k) c->ck_host[k] = cf * ph->h_m[k];
                h2d(c->d_Paf, paf, st);
                h2d(c->d_ck, c->ck_host, st);
            }
            FaceArgs fa;
            fa.faces = c->d_faces;
            fa.fmap = c->d_fmap;
            fa.face_out = c->d_face_out;
            fa.xyz = c->d_xyz;
            fa.v = d_v;
            fa.P_af = c->d_Paf;
            fa.aos = c->d_aos;
            fa.res = c->d_res;
            fa.rho = ph->rho;
            fa.beta = beta;
            fa.c_f = cf;
            for (int fc = 0; fc < S.n_fcolors; ++fc) {
                fa.F0 = S.fcolor_ptr[fc];
                fa.count = S.fcolor_ptr[fc + 1] - S.fcolor_ptr[fc];
                assemble_faces(fa, st);
            }
            add_traction((int)S.onode.size(), c->d_onode, c->d_oid, c->d_Paf, c->d_a_raw, c->d_res, st);
            // the host copies must outlive the asynchronous uploads
            HIPCHK(hipStreamSynchronize(st));
        }
        finalize_tangent(nnzb, c->d_rowof, c->d_col, c->d_mask, c->d_aos, c->sys[0].V64, st);
        finalize_rhs(S.N, c->d_mask, c->d_res, d_rhs, st);
        check_launch();
        c->c_f = cf;
        c->a_f = af;
        c->gamma_dt = gam * ph->dt;
        c->resistance_mode = resist;
        c->version++;
        c->sys[0].ready = c->sys[1].ready = false;
        c->assembled = true;
        return NS_OK;
    });
}

ns_status ns_nested_solve(ns_ctx* c, const ns_solve_opts* o, const double* d_rhs, double* d_x, ns_stats* hs,
                          hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() { return run_solve(c, 0, o, d_rhs, d_x, hs, st); });
}

ns_status ns_adjoint_solve(ns_ctx* c, const ns_solve_opts* o, const double* d_g, double* d_lambda, ns_stats* hs,
                           hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() { return run_solve(c, 1, o, d_g, d_lambda, hs, st); });
}

ns_status ns_newton_update(ns_ctx* c, double gamma_dt, const double* d_dx, double* d_y, double* d_ydot,
                           hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->bound) throw Fail{NS_ERR_STATE, "context not bound"};
        if (!d_dx || !d_y || !d_ydot) throw Fail{NS_ERR_ARG, "null argument"};
        newton_update(4 * (int64_t)c->sym.N, gamma_dt, d_dx, d_y, d_ydot, st);
        check_launch();
        return NS_OK;
    });
}

ns_status ns_time_step(ns_ctx* c, const ns_phys* phys, ns_outlet_model* om, const ns_newton_opts* nopt,
                       const ns_solve_opts* sopt, const double* d_y_n, const double* d_ydot_n, double* d_y,
                       double* d_ydot, ns_step_stats* hs, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->bound) throw Fail{NS_ERR_STATE, "context not bound"};
        if (!phys || !d_y_n || !d_ydot_n || !d_y || !d_ydot) throw Fail{NS_ERR_ARG, "null argument"};
        if (d_y == d_y_n || d_ydot == d_ydot_n || d_y == d_ydot) throw Fail{NS_ERR_ARG, "outputs alias inputs"};
        const Symbolic& S = c->sym;
        const int N = S.N, NO = S.n_out;
        const int64_t n4 = 4 * (int64_t)N;
        if (NO > 0 && (!om || !om->h_Rp || !om->h_C || !om->h_Rd || !om->h_Pd || !om->h_Pi || !om->h_P || !om->h_Q))
            throw Fail{NS_ERR_ARG, "outlet model missing"};
        for (int k = 0; k < NO; ++k)
            if (om->h_C[k] < 0 || (om->h_C[k] > 0 && !(om->h_Rd[k] > 0)))
                throw Fail{NS_ERR_ARG, "Windkessel needs C >= 0 and R_d > 0 when C > 0"};
        ns_newton_opts no{};
        if (nopt) no = *nopt;
        const double tol_R = dfltd(no.tol_R, 1e-6), tol_A = dfltd(no.tol_A, 1e-6);
        const double eps_abs = dfltd(no.eps_abs, 1e-8), eps_rel = dfltd(no.eps_rel, 1e-5);
        const int l_max = dflt(no.l_max, 20);
        const int nts = om ? dflt(om->n_ts, 100) : 100;
        const double am = 0.5 * (3.0 - phys->rho_inf) / (1.0 + phys->rho_inf);
        const double af = 1.0 / (1.0 + phys->rho_inf), gam = af;
        const double dt = phys->dt;
        ns_step_stats st_out{};
        auto t0 = std::chrono::steady_clock::now();
        HIPCHK(hipSetDevice(c->device));
        // predictor
        axpby<double>(n4, 1.0, d_y_n, 0.0, d_y_n, d_y, st);
        axpby<double>(n4, (gam - 1.0) / gam, d_ydot_n, 0.0, d_ydot_n, d_ydot, st);
        check_launch();
        std::vector<double> Qn(NO), Pn(NO), Pin(NO), Q(NO), P(NO), m(NO), Paf(NO);
        for (int k = 0; k < NO; ++k) {
            Qn[k] = om->h_Q[k];
            Pn[k] = om->h_P[k];
            Pin[k] = om->h_Pi[k];
        }
        auto flows = [&](const double* y) {
            if (NO == 0) return;
            ns_status r = ns_outlet_flow(c, y, Q.data(), st);
            if (r != NS_OK) throw Fail{r, c->err};
        };
        auto G = [&](int k, double q, double* pi_end) {
            return windkessel(om->h_Rp[k], om->h_C[k], om->h_Rd[k], om->h_Pd[k], Pin[k], Qn[k], q, nts, dt, pi_end);
        };
        ns_phys ph = *phys;
        ph.h_m = m.data();
        ph.h_P_af = Paf.data();
        ph.h_R = ph.h_P_n = ph.h_Q = nullptr;  // the reduced model gives m^k and P^k_{n+af}
        double r0 = 0.0, r = 0.0;
        bool conv = false;
        double asm_ms = 0.0, sol_ms = 0.0;
        // at most l_max corrector solves; the residual of the returned iterate
        // is always evaluated (assembly l_max + 1 when the solves run out)
        for (int l = 1; l <= l_max + 1; ++l) {
            flows(d_y);
            for (int k = 0; k < NO; ++k) {
                const double eps = std::max(eps_abs, eps_rel * std::fabs(Q[k]));
                P[k] = G(k, Q[k], nullptr);
                m[k] = (G(k, Q[k] + 0.5 * eps, nullptr) - G(k, Q[k] - 0.5 * eps, nullptr)) / eps;
                Paf[k] = (1.0 - af) * Pn[k] + af * P[k];
            }
            axpby<double>(n4, 1.0 - af, d_y_n, af, d_y, c->nt_yaf, st);
            axpby<double>(n4, 1.0 - am, d_ydot_n, am, d_ydot, c->nt_ydam, st);
            check_launch();
            auto ta = std::chrono::steady_clock::now();
            ns_status ra = ns_assemble_tangent(c, &ph, c->nt_yaf, c->nt_yaf + 3 * (int64_t)N, c->nt_ydam, c->nt_rhs,
                                               st);
            if (ra != NS_OK) throw Fail{ra, c->err};
            norm2<double>(n4, c->nt_rhs, c->nt_scal, c->d_red, st);
            check_launch();
            HIPCHK(hipMemcpyAsync(c->h_pinned, c->nt_scal, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            asm_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
            r = c->h_pinned[0];
            if (!std::isfinite(r)) throw Fail{NS_ERR_NAN, "residual is not finite"};
            if (l == 1) r0 = r;
            if (l - 1 < 32) st_out.res_hist[l - 1] = r;
            if (r <= tol_R * r0 || r <= tol_A) {
                conv = true;
                break;
            }
            if (l > l_max) break;
            ns_stats ls{};
            auto tsol = std::chrono::steady_clock::now();
            ns_status rs = ns_nested_solve(c, sopt, c->nt_rhs, c->nt_dx, &ls, st);
            sol_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tsol).count();
            if (rs < 0) throw Fail{rs, c->err};
            st_out.lin_outer += ls.outer_iters;
            st_out.lin_a += ls.a_iters;
            st_out.lin_s += ls.s_iters;
            st_out.lin_inner += ls.inner_iters;
            newton_update(n4, gam * dt, c->nt_dx, d_y, d_ydot, st);
            check_launch();
            st_out.iterations = l;
        }
        // reduced model at the accepted iterate
        flows(d_y);
        for (int k = 0; k < NO; ++k) {
            double pi_end = 0.0;
            const double pk = G(k, Q[k], &pi_end);
            om->h_Q[k] = Q[k];
            om->h_P[k] = pk;
            om->h_Pi[k] = pi_end;
        }
        HIPCHK(hipStreamSynchronize(st));
        st_out.converged = conv ? 1 : 0;
        st_out.res0 = r0;
        st_out.res = r;
        st_out.assemble_ms = asm_ms;
        st_out.solve_ms = sol_ms;
        st_out.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (hs) *hs = st_out;
        return conv ? NS_OK : NS_NOT_CONVERGED;
    });
}

ns_status ns_kernel_timing(ns_ctx* c, int32_t mask) {
    if (!c || mask < 0 || mask >= (1 << NS_KT_COUNT)) return NS_ERR_ARG;
    c->kt_mask = mask;
    return NS_OK;
}

ns_status ns_kernel_timing_period(ns_ctx* c, int32_t period) {
    if (!c || period < 1) return NS_ERR_ARG;
    c->kt_period = period;
    for (int i = 0; i < NS_KT_COUNT; ++i) c->kt_seen[i] = 0;
    return NS_OK;
}

ns_status ns_kernel_timing_read(ns_ctx* c, int32_t cls, double* out) {
    if (!c || !out || cls < 0 || cls >= NS_KT_COUNT) return NS_ERR_ARG;
    for (int i = 0; i < 3; ++i) {
        out[i] = c->kt_acc[cls][i];
        c->kt_acc[cls][i] = 0.0;
    }
    return NS_OK;
}

ns_status ns_query(const ns_ctx* c, int64_t* h) {
    if (!c || !h) return NS_ERR_ARG;
    h[0] = c->sym.N;
    h[1] = c->sym.g.nnz();
    h[2] = c->sym.shat.nnz();
    h[3] = c->sym.n_colors;
    h[4] = (int64_t)c->sym.onode.size();
    h[5] = (int64_t)c->sym.lv.size();
    return NS_OK;
}

ns_status ns_query_layout(const ns_ctx* c, int32_t* h) {
    if (!c || !h) return NS_ERR_ARG;
    h[0] = c->sym.ell;
    h[1] = c->sym.dcol.empty() ? 0 : 1;
    h[2] = c->bound && c->ell32 ? 1 : 0;
    h[3] = c->bound && c->col16 ? 1 : 0;
    return NS_OK;
}

ns_status ns_export_fixed_width_offsets(const ns_ctx* c, int16_t* h) {
    if (!c || !h || c->sym.ell == 0) return NS_ERR_ARG;
    std::copy(c->sym.dcol_ell.begin(), c->sym.dcol_ell.end(), h);
    return NS_OK;
}

ns_status ns_export_pattern(const ns_ctx* c, int32_t* rp, int32_t* col) {
    if (!c || !rp || !col) return NS_ERR_ARG;
    std::copy(c->sym.g.rp.begin(), c->sym.g.rp.end(), rp);
    std::copy(c->sym.g.col.begin(), c->sym.g.col.end(), col);
    return NS_OK;
}

ns_status ns_export_aggregates(const ns_ctx* c, int32_t level, int32_t* agg) {
    if (!c || !agg || level < 0 || level + 1 >= (int)c->sym.lv.size()) return NS_ERR_ARG;
    std::copy(c->sym.lv[level].agg.begin(), c->sym.lv[level].agg.end(), agg);
    return NS_OK;
}

ns_status ns_export_colors(const ns_ctx* c, int32_t* color) {
    if (!c || !color) return NS_ERR_ARG;
    std::copy(c->sym.color_of.begin(), c->sym.color_of.end(), color);
    return NS_OK;
}

ns_status ns_export_bsr(ns_ctx* c, int32_t transposed, double* d_dst, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->assembled) throw Fail{NS_ERR_STATE, "no tangent assembled"};
        if (!d_dst) throw Fail{NS_ERR_ARG, "null argument"};
        if (transposed) ensure_transposed(c, st);
        export_aos(c->sym.g.nnz(), c->sys[transposed ? 1 : 0].V64, d_dst, st);
        check_launch();
        HIPCHK(hipStreamSynchronize(st));
        return NS_OK;
    });
}

ns_status ns_export_shat(ns_ctx* c, int32_t* rp, int32_t* col, double* d_val, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->assembled) throw Fail{NS_ERR_STATE, "no tangent assembled"};
        if (rp) std::copy(c->sym.shat.rp.begin(), c->sym.shat.rp.end(), rp);
        if (col) std::copy(c->sym.shat.col.begin(), c->sym.shat.col.end(), col);
        if (d_val) {
            setup_system(c, c->sys[0], false, st);
            HIPCHK(hipMemcpyAsync(d_val, c->sys[0].shat64, c->sym.shat.nnz() * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        return NS_OK;
    });
}

ns_status ns_export_outlet_vectors(ns_ctx* c, double* d_a, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->bound) throw Fail{NS_ERR_STATE, "context not bound"};
        const int N = c->sym.N;
        for (int k = 0; k < c->sym.n_out; ++k) {
            fill<double>(3 * (int64_t)N, 0.0, d_a + 3 * (int64_t)N * k, st);
        }
        // scatter slots into dense vectors (host loop over slots; tiny)
        std::vector<double> a(3 * c->sym.onode.size());
        if (!a.empty())
            HIPCHK(hipMemcpyAsync(a.data(), c->d_a_msk, a.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (size_t sl = 0; sl < c->sym.onode.size(); ++sl) {
            const int k = c->sym.oid[sl];
            HIPCHK(hipMemcpyAsync(d_a + 3 * (int64_t)N * k + 3 * (int64_t)c->sym.onode[sl], &a[3 * sl],
                                  3 * sizeof(double), hipMemcpyHostToDevice, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        return NS_OK;
    });
}

ns_status ns_apply(ns_ctx* c, int32_t op, const ns_solve_opts* opts, const double* d_x, double* d_y,
                   hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    return guard(c, [&]() -> ns_status {
        if (!c->assembled) throw Fail{NS_ERR_STATE, "no tangent assembled"};
        if (!d_x || !d_y) throw Fail{NS_ERR_ARG, "null argument"};
        HIPCHK(hipSetDevice(c->device));
        HIPCHK(hipStreamSynchronize(st));
        st = c->own;
        Ctl K{};
        K.c = c;
        K.st = st;
        if (opts) K.o = *opts;
        K.o.atol = K.o.atol > 0 ? K.o.atol : 1e-50;
        K.sc.replay = K.o.h_sched;
        K.sc.replay_len = K.o.sched_len;
        K.sy = &c->sys[0];
        const bool f32 = K.o.precision == NS_FP32_INNER;
        setup_system(c, c->sys[0], f32, st);
        upload_coef(c, c->sys[0], K.o, st);
        const int N = c->sym.N;
        const int64_t nin[] = {4L * N, 3L * N, N, 3L * N, N, N, 3L * N, N, N, 4L * N, 3L * N, 4L * N};
        const int64_t nout[] = {4L * N, 3L * N, 3L * N, N, N, N, 3L * N, N, N, 4L * N, 3L * N, 4L * N};
        if (op < 0 || op > NS_OP_PSIMPLE) throw Fail{NS_ERR_ARG, "unknown operator"};
        check_solve_opts(K.o);
        auto run = [&](auto tag) {
            using T = decltype(tag);
            Nested<T> P(K);
            const T* x;
            T* y;
            if (std::is_same<T, double>::value) {
                x = reinterpret_cast<const T*>(d_x);
                y = reinterpret_cast<T*>(d_y);
            } else {
                convert<double, T>(nin[op], d_x, as<T>(c->t_s), st);
                x = as<T>(c->t_s);
                y = as<T>(c->t_r4);
            }
            switch (op) {
                case NS_OP_FULL: {
                    RankOne<T> r = P.rank_one();
                    if (r.slot_of)
                        outlet_dot<T>(c->sym.n_out, c->d_optr, c->d_onode, Typed<T>::amsk(c), Typed<T>::ck(c), x,
                                      as<T>(c->d_s), st);
                    spmv_full<T>(N, c->d_rp, c->d_col, P.V(), P.plane(), x, y, T(1), nullptr, T(0),
                                 r.slot_of ? &r : nullptr, st, P.ell(), P.dcol_planes());
                    break;
                }
                case NS_OP_A: P.applyA(x, y); break;
                case NS_OP_B: spmv<T>(3, 1, P.op(0, 3), x, y, T(1), nullptr, T(0), nullptr, nullptr, st); break;
                case NS_OP_C: spmv<T>(1, 3, P.op(3, 0), x, y, T(1), nullptr, T(0), nullptr, nullptr, st); break;
                case NS_OP_D: spmv<T>(1, 1, P.op(3, 3), x, y, T(1), nullptr, T(0), nullptr, nullptr, st); break;
                case NS_OP_SHAT: {
                    BlockOp<T> M = P.level_op(c->sys[0].S[0]);
                    spmv<T>(1, 1, M, x, y, T(1), nullptr, T(0), nullptr, nullptr, st);
                    break;
                }
                case NS_OP_VCYCLE_A: P.vcycle(c->sys[0].A, 0, x, y); break;
                case NS_OP_VCYCLE_S: P.vcycle(c->sys[0].S, 0, x, y); break;
                case NS_OP_SCHUR: P.schur(x, y); break;
                case NS_OP_PSCR: P.scr(x, y); break;
                case NS_OP_SOLVE_A: P.solveA(x, y, dfltd(K.o.rtol_A, 1e-3)); break;
                case NS_OP_PSIMPLE: P.simple(x, y); break;
            }
            if (!std::is_same<T, double>::value) convert<T, double>(nout[op], y, d_y, st);
        };
        if (f32) run(float{});
        else run(double{});
        check_launch();
        HIPCHK(hipStreamSynchronize(st));
        timing_collect(c);
        if (K.o.h_sched_out)
            for (int i = 0; i < (int)K.sc.log.size() && i < K.o.sched_cap; ++i) K.o.h_sched_out[i] = K.sc.log[i];
        return NS_OK;
    });
}

}  // extern "C"
