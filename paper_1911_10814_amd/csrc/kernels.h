// Launch wrappers of the HIP kernels (internal).
#pragma once

#include "internal.h"

namespace ns {

constexpr int kBlock = 256;
constexpr int kMaxRedBlocks = 1024;

// Rank-one epilogue of the A-operator: y_i += s_k a^k_i for outlet slots.
template <typename T>
struct RankOne {
    const int32_t* slot_of = nullptr;  // [N] slot of node or -1
    const int32_t* oid = nullptr;      // [slots] outlet of slot
    const T* aval = nullptr;           // [slots][3]
    const T* s = nullptr;              // [n_out] c_k (a^k . x)
};

// Optional epilogue of an operator application y = M x that also performs the
// first Chebyshev step of the V-cycle which follows on y, from a zero guess:
// x0 = d0 = coef[0] * dinv .* y.
template <typename T>
struct FirstStep {
    const T* dinv = nullptr;
    const T* coef = nullptr;
    T* x = nullptr;
    T* d = nullptr;
};

// Block-sparse operator: rows of BR, columns of BC unknowns; value of block k
// at (r, c) is v[r*rs + c*cs + k].
template <typename T>
struct BlockOp {
    int n = 0;
    const int32_t* rp = nullptr;
    const int32_t* col = nullptr;
    const T* v = nullptr;
    int64_t rs = 0, cs = 0;
    const T* dextra = nullptr;  // optional extra diagonal [BR*n]
    const int16_t* dcol = nullptr;  // when set, column of block k of row i is i + dcol[k] (col is not read)
    int ell = 0;  // > 0: fixed-width rows, row i's blocks at i*ell + l (l < ell; zero blocks pad), rp not read
    int lanes = 16;             // lanes per block row (8, 16, 32 or 64), from the mean row length
    int unroll = 2;             // 4- and 8-lane rows: 16 (2) or 32 (4) entries per trip, from the mean row length
    int xcd = 0;                // 1: each XCD takes one contiguous range of rows (xcd_block)
};

// Kernel timing: the next launch of the block-SpMV family (spmv, spmv_full,
// cheb_step) records `start` and `stop` at its own start and end; returns to
// plain launches after that one.  launch_events_pending() tells whether the
// events are still unused.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_pending();

// Lanes per row for a pattern with nnz blocks of bs x bs values over n rows.
// Blocks of 3x3 values: one pass over a typical row, so consecutive rows give
// contiguous loads across the wavefront.  Scalar rows (S_hat levels, 1 value
// per entry): 8 lanes whatever the row length, each with several entries in
// flight (a level-1 S_hat smoothing step on the 4e6-node contraction-expansion,
// ~44 entries per row: 160 us with 8 lanes against 178 / 258 / 335 us with 16 /
// 32 / 64).
inline int lanes_for(int64_t nnz, int n, int bs) {
    if (bs == 1) return 8;
    const double avg = n > 0 ? (double)nnz / n : 0.0;
    return avg <= 16.0 ? 16 : (avg <= 32.0 ? 32 : 64);
}
// Entries per trip of a 4- or 8-lane row walk (2: 16 entries, 4: 32): enough
// that a typical row is one trip (all its loads in flight together).
inline int unroll_for(int64_t nnz, int n) { return (double)nnz <= 16.0 * (n > 0 ? n : 1) ? 2 : 4; }

// y = alpha * (M x [+ dextra x] [+ rank one]) + beta * z, then y *= rscale
template <typename T>
void spmv(int br, int bc, const BlockOp<T>& M, const T* x, T* y, T alpha, const T* z, T beta,
          const T* rscale, const RankOne<T>* ro, hipStream_t st, const FirstStep<T>* fs = nullptr);

// Full 4x4 field-split operator: y = alpha [A B; C D] x + beta z.
template <typename T>
void spmv_full(int n, const int32_t* rp, const int32_t* col, const T* V, int64_t nnzb, const T* x, T* y,
               T alpha, const T* z, T beta, const RankOne<T>* ro, hipStream_t st, int ell = 0,
               const int16_t* dcol_ell = nullptr);

// s[k] = c[k] * sum_{slots of k} a . x
template <typename T>
void outlet_dot(int n_out, const int32_t* optr, const int32_t* onode, const T* aval, const T* c, const T* x,
                T* s, hipStream_t st);

template <typename T>
void axpby(int64_t n, T a, const T* x, T b, const T* y, T* out, hipStream_t st);  // out = a x + b y
template <typename Tin, typename Tout>
void convert(int64_t n, const Tin* x, Tout* y, hipStream_t st);
template <typename T>
void fill(int64_t n, T val, T* y, hipStream_t st);
template <typename T>
void mul(int64_t n, const T* a, const T* x, T* y, hipStream_t st);  // y = a .* x

// One CGS2 Arnoldi step: w (= V_{j+1}, holding P^{-1} M v_j) is orthogonalised
// against V_0..V_j by two classical Gram-Schmidt passes, the Hessenberg
// column j and Givens rotation are updated on the device (status[0] =
// |g_{j+1}|, [1] = breakdown flag, [2] = 1/h_{j+1,j}, [3] = ||w_pre||), and
// w is normalised.  h1 [j+2] / h2 [j+1] receive the dot products of the two
// passes (h1[j+1] = ||w_pre||^2); `red` holds the per-block partial sums.
// Bases of up to this many vectors take the single-pass form of the pass-1
// update and pass-2 dots (each thread's packs of the basis kept in registers).
constexpr int kOrthFuseMax = 16;
struct GivensArgs {
    int j = 0, ldh = 0;
    const double* h1 = nullptr;
    const double* h2 = nullptr;
    double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *status = nullptr;
    double* hstatus = nullptr;  // optional host-mapped copy of status[0..1]
    // optional host-mapped step number, stored (system-scope release) after
    // hstatus, so that the host can see the step's status without waiting for
    // the end of the kernel
    unsigned long long* hseq = nullptr;
    unsigned long long seq = 0;
};
template <typename T>
void arnoldi_cgs2(int64_t n, int j, const T* V, int64_t ldv, T* w, double* h1, double* h2, const GivensArgs& ga,
                  double* red, hipStream_t st);
void backsolve(int k, int ldh, const double* H, const double* g, double* y, hipStream_t st);
void init_g(double* g, int len, double beta, hipStream_t st);  // g = [beta, 0, ...]
// v /= nrm[0]; g = [nrm[0], 0, ...] (len entries)
template <typename T>
void start_cycle(int64_t n, T* v, const double* nrm, double* g, int len, hipStream_t st);
// x = (accumulate ? x : 0) + sum_i V_i y_i
template <typename T, typename TX>
void combine(int64_t n, int k, const T* V, int64_t ldv, const double* y, TX* x, bool accumulate,
             hipStream_t st);
// out[0] = ||x|| (device); also hout[0] (host-mapped) when not null
template <typename T>
void norm2(int64_t n, const T* x, double* out, double* red, hipStream_t st, double* hout = nullptr);
template <typename T>
void scale_by(int64_t n, const T* x, const double* s, bool inverse, T* y, hipStream_t st);

// AMG kernels
// Chebyshev coefficients in device memory: coef[0] = 1/theta; step s >= 1
// uses (c1, c2) = (coef[2s-1], coef[2s]).
constexpr int kMaxChebDegree = 8;
constexpr int kCoefLen = 2 * kMaxChebDegree;
// the last slot of a level's coefficient array holds the scaling of the
// coarse-grid correction that level receives from the next one
constexpr int kCoefScale = kCoefLen - 1;
static_assert(2 * (kMaxChebDegree - 1) < kCoefScale, "Chebyshev step coefficients overlap the scale slot");
template <typename T>
void cheb_first(int64_t n, const T* b, const T* dinv, const T* coef, T* x, T* d, hipStream_t st);
template <typename T>
void cheb_step(int bs, const BlockOp<T>& M, const T* xin, T* xout, T* d, const T* b, const T* dinv, const T* coef,
               int step, const int32_t* agg, const T* ec, hipStream_t st);
// scale (device scalar, or nullptr for 1) multiplies the restricted right-hand
// side, i.e. the coarse-grid correction the coarse cycle returns
template <typename T>
void restrict_first(int nc, int bs, const int32_t* aptr, const int32_t* anodes, const T* r, T* bc, T* xc, T* dc,
                    const T* dinvc, const T* coefc, const T* scale, hipStream_t st);
// Factored S_hat = D - C diag(A)^{-1} B on the node pattern (V: the 16 value
// planes; t: [4n] scratch, 16-byte aligned; columns from dcol as in BlockOp
// when it is set, else from col).  With coef == nullptr: y = alpha S_hat xx + beta z;
// else one Chebyshev step y = xx + d, d = c1 d + c2 dinv (b - S_hat xx), where
// xx = x, or x + P ec when agg != nullptr.
template <typename T>
void shat_factored(int n, const int32_t* rp, const int32_t* col, const int16_t* dcol, int ell, const T* V,
                   int64_t nnzb, const T* dinvA, const T* x, const int32_t* agg, const T* ec, T* t, T* y, T alpha,
                   const T* z, T beta, const T* b, const T* dinv, const T* coef, int step, T* d, int xcd, int lanes,
                   hipStream_t st);
// Planes of a node-graph matrix (p planes of nnzb values, row pointers rp)
// converted into the fixed-width row layout (p planes of n*ell values, row
// i's blocks at i*ell + l, zero past the row's end).
template <typename Tin, typename Tout>
void to_ell(int n, int ell, const int32_t* rp, const Tin* src, int64_t nnzb, int planes, Tout* dst, hipStream_t st);
// bc = P^T (b - M x) in one launch (residual rows summed per aggregate), plus
// the coarse first Chebyshev step when xc != nullptr (as restrict_first)
template <typename T>
void resid_restrict(int bs, const BlockOp<T>& M, const T* x, const T* b, int nc, const int32_t* aptr,
                    const int32_t* anodes, T* bc, T* xc, T* dc, const T* dinvc, const T* coefc, const T* scale,
                    hipStream_t st);
template <typename T>
void restrict_agg(int nc, int bs, const int32_t* aptr, const int32_t* anodes, const T* r, T* bc, hipStream_t st);
template <typename T>
void prolong_add(int n, int bs, const int32_t* agg, const T* ec, T* x, hipStream_t st);
template <typename T>
void dense_gemv(int n, const double* Minv, const T* b, T* x, hipStream_t st);

// Set-up kernels (FP64)
void galerkin(int64_t nq, int np_r, int np_c, const int32_t* gptr, const int32_t* gidx, const double* vf,
              int64_t frs, int64_t fcs, double* vc, int64_t crs, int64_t ccs, const int32_t* qrow,
              const int32_t* ccol, const double* dextra, const int32_t* aptr, const int32_t* anodes,
              hipStream_t st);
void block_dinv(int n, int bs, const int32_t* rp, const int32_t* col, const double* v, int64_t rs, int64_t cs,
                const double* dextra, double* dinv, double* diag, hipStream_t st);
void shat_numeric(int n, const int32_t* rp, const int32_t* col, const double* V, int64_t nnzb,
                  const double* dinvA, const int32_t* srp, const int32_t* scol, double* shat, hipStream_t st);
// inv_i = (left half of work_i)^{-1} by Gauss-Jordan with partial pivoting on
// [M_i | I] for two independent matrices, one launch per pivot step for both;
// work_i holds [2][n_i][2 n_i]: the input [M_i | I] in the first half, the
// second half is the ping-pong buffer (both overwritten)
void gauss_jordan_inverse2(int n0, double* work0, double* inv0, int n1, double* work1, double* inv1,
                           hipStream_t st);
void dense_from_csr(int nb, int bs, const int32_t* rp, const int32_t* col, const double* v, int64_t rs,
                    int64_t cs, const double* dextra, double* work, hipStream_t st);
// out[0] = max_r |dinv_r| sum_c |M_rc| (Gershgorin bound of D^{-1} M);
// part: scratch of ceil(n * M.lanes / kBlock) doubles
void gershgorin_bound(const BlockOp<double>& M, int bs, const double* dinv, double* part, double* out,
                      hipStream_t st);
void power_start(int64_t n, double* x, hipStream_t st);
void rank_one_diag(int n_slots, const int32_t* onode, const int32_t* oid, const double* amsk, const double* ck,
                   double* dK, hipStream_t st);
void transpose_values(int64_t nnzb, const int32_t* tmap, const double* V, double* Vt, hipStream_t st);
void export_aos(int64_t nnzb, const double* V, double* dst, hipStream_t st);

// Assembly
struct AsmArgs {
    int E0 = 0, count = 0;            // element range of one colour
    const int32_t* tets = nullptr;    // [E][4] (sorted by colour)
    const int32_t* emap = nullptr;    // [E][16]
    const double* xyz = nullptr;
    const double* v = nullptr;
    const double* p = nullptr;
    const double* vdot = nullptr;
    double* aos = nullptr;            // [nnzb][16]
    double* res = nullptr;            // [4N]
    int N = 0;
    double rho = 0, mu = 0, dt = 0, c_m = 0, c_f = 0, c_t = 0, c_i = 0;
};
void assemble_elements(const AsmArgs& a, hipStream_t st);
struct FaceArgs {
    int F0 = 0, count = 0;
    const int32_t* faces = nullptr;   // [F][3]
    const int32_t* fmap = nullptr;    // [F][9]
    const int32_t* face_out = nullptr;
    const double* xyz = nullptr;
    const double* v = nullptr;
    const double* P_af = nullptr;     // [n_out] device
    double* aos = nullptr;
    double* res = nullptr;
    double rho = 0, beta = 0, c_f = 0;
};
void assemble_faces(const FaceArgs& a, hipStream_t st);
void outlet_vectors(int F0, int count, const int32_t* faces, const int32_t* fslot, const double* xyz,
                    double* a_raw, hipStream_t st);
void mask_outlet(int n_slots, const int32_t* onode, const uint8_t* mask, const double* a_raw, double* a_msk,
                 hipStream_t st);
void finalize_tangent(int64_t nnzb, const int32_t* row_of, const int32_t* col, const uint8_t* mask,
                      const double* aos, double* V, hipStream_t st);
void finalize_rhs(int N, const uint8_t* mask, const double* res, double* rhs, hipStream_t st);
// res[3 node + c] += P_af[outlet] a^k_{node,c}  (traction term of the outlets)
void add_traction(int n_slots, const int32_t* onode, const int32_t* oid, const double* P_af, const double* a_raw,
                  double* res, hipStream_t st);
void newton_update(int64_t n, double gdt, const double* dx, double* y, double* ydot, hipStream_t st);
// Largest outlet count of ns_resistance_gradient_noalloc: its file-scope
// scratch holds two dot products per outlet (64 KiB).
constexpr int kNoAllocMaxOutlets = 4096;
// device address of that scratch on `device` (the current device), looked up once per device
hipError_t noalloc_scratch(int device, double** out);
// resistance outlets: ck = c_f R, P_af = (1 - af) P_n + af R Q (P_n == nullptr: R Q)
void resistance_outlets(int n_out, const double* R, const double* P_n, const double* Q, double af, double cf,
                        double* ck, double* P_af, hipStream_t st);
// grad[k] = -s_lam[k] (af Q[k] + cf s_x[k])
void resistance_grad(int n_out, const double* s_lam, const double* s_x, const double* Q, double af, double cf,
                     double* grad, hipStream_t st);

}  // namespace ns
