// Internal declarations of the nested block solver library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "ns_api.h"

namespace ns {

// ---------------------------------------------------------------------------
// Host-side symbolic structures (built once per mesh in ns_ctx_create)
// ---------------------------------------------------------------------------

struct Csr {
    int n = 0;
    std::vector<int32_t> rp, col;  // sorted columns, diagonal included
    int64_t nnz() const { return (int64_t)col.size(); }
};

struct AmgLevelSym {
    int n = 0;            // nodes at this level
    Csr a;                // pattern of the A-hierarchy operator (3x3 blocks)
    Csr s;                // pattern of the S_hat-hierarchy operator (scalars)
    std::vector<int32_t> a_qrow;  // row of every nnz of `a` (levels >= 1)
    // aggregation to the next level (empty on the coarsest level)
    std::vector<int32_t> agg;            // node -> coarse node
    std::vector<int32_t> aptr, anodes;   // coarse node -> its fine nodes (CSR)
    // Galerkin gather lists of THIS level's operators from the finer level:
    // coarse nnz q sums fine nnz gidx[gptr[q] .. gptr[q+1])
    std::vector<int32_t> gptr, gidx;     // A hierarchy
    std::vector<int32_t> sgptr, sgidx;   // S_hat hierarchy
};

struct Symbolic {
    int N = 0, E = 0, n_out = 0, F = 0;
    Csr g;                               // node graph = BSR pattern
    std::vector<int16_t> dcol;           // [nnzb] col - row when every |col - row| <= 32767, else empty
    // fixed-width rows for the FP32 planes: ell = the longest row (<= 16, and
    // dcol available), row i's blocks at i*ell + l, padded with zero blocks
    // whose offset is 0; 0 when the pattern does not allow it
    int ell = 0;
    std::vector<int16_t> dcol_ell;       // [N*ell] column offsets in that layout
    std::vector<int32_t> diag_pos;       // [N]
    std::vector<int32_t> row_of;         // [nnzb]
    std::vector<int32_t> tmap;           // [nnzb] index of the transposed block
    // elements sorted by colour
    int n_colors = 0;
    std::vector<int32_t> color_ptr;      // [n_colors+1]
    std::vector<int32_t> elem_perm;      // sorted position -> original element
    std::vector<int32_t> tets;           // [E][4] in sorted order
    std::vector<int32_t> emap;           // [E][16] block index of pair (a,b) = a*4+b
    std::vector<int32_t> color_of;       // [E] colour of each original element
    // outlets
    std::vector<int32_t> onode;          // [n_onodes] node of each outlet slot
    std::vector<int32_t> oid;            // [n_onodes] outlet of each slot
    std::vector<int32_t> optr;           // [n_out+1] slot ranges per outlet
    std::vector<int32_t> slot_of;        // [N] slot of node or -1
    int n_fcolors = 0;
    std::vector<int32_t> fcolor_ptr;
    std::vector<int32_t> faces;          // [F][3] sorted by colour
    std::vector<int32_t> face_out;       // [F] outlet of each face
    std::vector<int32_t> fmap;           // [F][9] block index of pair (a,b) = a*3+b
    std::vector<int32_t> fslot;          // [F][3] slot of each face node
    // S_hat pattern (distance-2 node graph)
    Csr shat;
    // AMG hierarchy (level 0 = fine)
    std::vector<AmgLevelSym> lv;
};

std::string build_symbolic(const ns_mesh* mesh, const ns_ctx_opts& o, Symbolic& S);

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------

struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return base ? p : nullptr;
    }
};

struct AmgLevelDev {
    int n = 0, bs = 0;
    // pattern (device)
    int32_t *rp = nullptr, *col = nullptr;
    int64_t nnz = 0;
    // numeric values: planes [bs*bs][nnz] (level 0 of the A hierarchy points
    // into the tangent storage instead)
    double* v64 = nullptr;
    float* v32 = nullptr;
    int64_t rstride = 0, cstride = 0;   // plane strides between block rows / columns
    double* dinv64 = nullptr;
    float* dinv32 = nullptr;
    const double* dextra64 = nullptr;   // extra diagonal (level 0 of A: lumped diag K)
    const float* dextra32 = nullptr;
    double lmax = 0.0;
    double* coef64 = nullptr;           // Chebyshev step coefficients (device)
    float* coef32 = nullptr;
    // Galerkin gather lists from the finer level (levels >= 1)
    int32_t *gptr = nullptr, *gidx = nullptr, *qrow = nullptr;
    // restriction/prolongation to the next level
    int32_t *agg = nullptr, *aptr = nullptr, *anodes = nullptr;
    // work vectors (sized for FP64, reused for FP32): x0, x1, d, r, b
    double *x0 = nullptr, *x1 = nullptr, *d = nullptr, *r = nullptr, *b = nullptr;
    // coarsest level: dense inverse [n*bs][n*bs] FP64 and its work matrices
    // (two halves of [M | I], [2][n*bs][2*n*bs])
    double* inv = nullptr;
    double* work = nullptr;
};

struct SystemDev {
    // tangent in SoA planes [16][nnzb] (plane 4r+c; r,c = u,v,w,p)
    double* V64 = nullptr;
    float* V32 = nullptr;
    double *dK64 = nullptr, *diagA64 = nullptr, *dinvA64 = nullptr;  // [3N]
    float *dK32 = nullptr, *dinvA32 = nullptr;
    double* shat64 = nullptr;  // [nnz S_hat]
    float* shat32 = nullptr;
    std::vector<AmgLevelDev> A, S;   // hierarchies
    int coef_deg = 0;                // number of Chebyshev steps the device coefficients cover
    double coef_ratio = 0.0;         // and the interval ratio
    double coef_scale[2] = {0.0, 0.0};  // and the coarse-grid correction scales (A, S_hat)
    bool ready = false;              // per-step set-up done for the current tangent
    bool have32 = false;
    uint64_t version = 0;            // tangent version the set-up belongs to
};

struct KrylovWs {
    int m = 0;
    int64_t n = 0;
    int64_t ld = 0;         // row stride of V and Z: n rounded up to 64 elements
    double* V = nullptr;    // [(m+1)][ld] (FP64 size; reused as FP32 with the same ld)
    double* Z = nullptr;    // [m][ld] (outer level only)
    double* tmp = nullptr;  // [n]
    double* H = nullptr;    // [(m+1)*m] column-major, leading dim m+1
    double* cs = nullptr;
    double* sn = nullptr;
    double* g = nullptr;    // [m+1]
    double* y = nullptr;    // [m]
    double* h = nullptr;    // [2][m+2] dot results of the two CGS passes (FP64 or FP32)
    double* status = nullptr;  // [4]: |g_{j+1}|, breakdown flag, 1/h_{j+1,j}, ||w_pre||
};

}  // namespace ns

struct ns_ctx {
    ns::Symbolic sym;
    ns_ctx_opts opts{};
    std::string err;
    size_t ws_bytes = 0;
    bool bound = false;
    int device = -1;
    // device copies of the symbolic data
    int32_t *d_rp = nullptr, *d_col = nullptr, *d_diag = nullptr, *d_rowof = nullptr, *d_tmap = nullptr;
    int16_t* d_dcol = nullptr;   // 16-bit column offsets of the node graph (null when they do not fit)
    int16_t* d_dcol_ell = nullptr;  // the same in the fixed-width row layout (null without one)
    int32_t *d_tets = nullptr, *d_emap = nullptr;
    int32_t *d_faces = nullptr, *d_fmap = nullptr, *d_fslot = nullptr, *d_face_out = nullptr;
    int32_t *d_onode = nullptr, *d_oid = nullptr, *d_slot_of = nullptr, *d_optr = nullptr;
    double* d_Paf = nullptr;     // [n_out] outlet pressures of the last assembly
    int32_t *d_srp = nullptr, *d_scol = nullptr;
    uint8_t* d_mask = nullptr;
    double* d_xyz = nullptr;
    double* d_a_raw = nullptr;   // [n_onodes][3] a^k (Dirichlet entries kept)
    double* d_a_msk = nullptr;   // [n_onodes][3] a^k with Dirichlet entries zeroed
    float* d_a_msk32 = nullptr;
    double* d_aos = nullptr;     // [nnzb][16] assembly accumulator
    double* d_res = nullptr;     // [4N] residual accumulator
    double* d_ck = nullptr;      // [n_out] rank-one weights c_k = alpha_f gamma dt m^k
    float* d_ck32 = nullptr;
    double* d_s = nullptr;       // [n_out] rank-one dot results
    double* d_s2 = nullptr;      // [n_out] second dot buffer (gradient contraction)
    double* d_R = nullptr;       // [n_out] resistances of the last resistance-mode assembly
    double* d_Pn = nullptr;      // [n_out] its P^k_n
    double* d_Q = nullptr;       // [n_out] its outlet flows Q^k
    double* d_grad = nullptr;    // [n_out] dL/dR of ns_resistance_gradient
    double* noalloc_scratch = nullptr;  // device address of the allocation-free variant's scratch
    double* d_red = nullptr;     // reduction partials
    ns::SystemDev sys[2];        // 0: forward, 1: transposed
    ns::KrylovWs kw_out, kw_A, kw_S;
    // P_SCR / Algorithm 2 temporaries (FP64-sized)
    double *t_s = nullptr, *t_yhat = nullptr, *t_tp = nullptr, *t_yp = nullptr, *t_tv = nullptr,
           *t_yv = nullptr, *t_xhat = nullptr, *t_xbar = nullptr, *t_xt = nullptr, *t_r4 = nullptr;
    double* t_sf = nullptr;  // [3N] scratch of the factored S_hat application
    double* t_ps = nullptr;  // [2N] residual and correction of the P_S iteration
    // time step: state at n+af / n+am, residual, Newton correction [4N], scalars
    double *nt_yaf = nullptr, *nt_ydam = nullptr, *nt_rhs = nullptr, *nt_dx = nullptr, *nt_scal = nullptr;
    double* d_bnd = nullptr; // [2 hierarchies][levels][3] smoother-bound scalars
    double* h_pinned = nullptr;  // pinned host scalars
    double* h_mapped = nullptr;  // pinned, device-mapped host scalars written by kernels
    double* d_mapped = nullptr;  // device address of h_mapped
    unsigned long long step_seq = 0;     // numbers the Arnoldi steps whose status the host reads
    unsigned long long slot_seq[2] = {};  // step number expected in each status slot (0: wait for the stream)
    std::vector<double> h_xyz;   // host copies uploaded by ns_ctx_bind
    std::vector<uint8_t> h_mask;
    uint64_t version = 0;        // incremented by every assembly
    bool assembled = false;
    double c_f = 0.0;            // alpha_f gamma dt of the last assembly
    double a_f = 0.0;            // alpha_f and gamma dt of the last assembly
    double gamma_dt = 0.0;
    bool resistance_mode = false;  // the last assembly took resistance outlets (ns_phys.h_R)
    // kernel timing (HIP event pairs around launches of selected classes)
    int32_t kt_mask = 0;
    int32_t kt_period = 1;                   // bracket every kt_period-th launch of a timed class
    uint64_t kt_seen[NS_KT_COUNT] = {};      // launches of each class since the period was set
    std::vector<hipEvent_t> kt_ev;           // pool: 2 events per timed launch
    std::vector<std::pair<int, double>> kt_pending;  // (class, bytes) per used pair
    double kt_acc[NS_KT_COUNT][3] = {{0}};   // per class: launches, ms, bytes
    // library-owned stream (solves run here; graph capture needs a non-default stream)
    hipStream_t own = nullptr;
    hipEvent_t step_ev[2] = {nullptr, nullptr};  // completion of queued Arnoldi steps
    // set-up: the smoother-bound chains of the AMG levels run on auxiliary
    // streams (default priority) beside the coarsest inverses on `own`
    static constexpr int kAux = 4;
    hipStream_t aux[kAux] = {};
    hipEvent_t aux_ev[kAux] = {};
    hipEvent_t fork_ev = nullptr;
    bool use_graphs = true;
    int xcd_mode = -1;           // XCD-contiguous row ranges: -1 by size, 0 off, 1 on
    int prolong_mode = -1;       // finest A prolongation: -1 by size, 0 fused into smoothing, 1 separate pass
    int unroll_mode = -1;        // 4- and 8-lane row walks: -1 by mean row length, else 2 or 4 (16 or 32 per trip)
    bool col16 = false;          // finest-level products read the 16-bit column offsets
    bool ell32 = false;          // the FP32 tangent planes are stored in the fixed-width row layout
    // captured Arnoldi steps, (kind, system, precision, pc_A, pc_I, degrees, cycles_S, j), and
    // set-up chains, (set-up kind, system, 0 ..., chain) -> executable graph
    using GraphKey = std::tuple<int, int, int, int, int, int, int, int, int>;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<double> ck_host;
    std::vector<double> h_outlets;   // host staging of R, P_n, Q for the asynchronous uploads
};
