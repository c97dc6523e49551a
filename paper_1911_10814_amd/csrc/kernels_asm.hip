// Tangent and residual assembly of one Newton step on gfx950.
//
// Volume terms (Sec. 2.3, residual-based VMS forms B_m^vol and B_p with
// tau_M, tau_C and the metric G built with the simplex matrix M) are
// integrated with the 4-point degree-2 rule; the tangent blocks are the
// alpha_m / alpha_f gamma dt weighted derivatives of Sec. 2.5 with tau_M and
// tau_C held at the current state.  Sixteen lanes per element, one per
// (a, b) node pair, and one launch per colour (no two elements of a colour
// share a node), so every block and residual entry is updated by plain
// read-modify-write without atomics.  The
// blocks are accumulated as [nnzb][16] (128 contiguous bytes per block hit)
// and transposed into the [16][nnzb] value planes the solver streams.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace ns {

namespace {
inline unsigned grid_for(int64_t t) { return (unsigned)((t + kBlock - 1) / kBlock); }

// barycentric coordinates of the 4-point rule: (qa, qb, qb, qb) and permutations
#define QA 0.58541019662496845446  // (5 + 3 sqrt 5) / 20
#define QB 0.13819660112501051518  // (5 - sqrt 5) / 20
__device__ inline double nq(int q, int a) { return q == a ? QA : QB; }
}  // namespace

// One element per 16 lanes, one lane per (a, b) node pair: each lane
// recomputes the element's geometry and quadrature-point state (cheap next to
// a tangent block, and it keeps every array in registers with no
// lane-dependent indexing), accumulates the (a, b) block over the four points
// and, in lane (a, 0), the residual of node a.  The 16 lanes of an element
// touch 16 distinct blocks and lanes (a, 0) four distinct residual rows, so the
// colouring still makes every update race-free.
constexpr int kPairs = 16;

__device__ inline double pick(int a, double x0, double x1, double x2, double x3) {
    return a == 0 ? x0 : a == 1 ? x1 : a == 2 ? x2 : x3;
}

__global__ __launch_bounds__(kBlock) void k_assemble_elements(AsmArgs g) {
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (tid >= (int64_t)kPairs * g.count) return;
    const int64_t s = g.E0 + tid / kPairs;
    const int pair = (int)(tid % kPairs), a = pair >> 2, b = pair & 3;
    int t[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) t[c] = g.tets[4 * s + c];
    double X[4][3];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) X[c][i] = g.xyz[3 * (int64_t)t[c] + i];
    double e[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) e[k][i] = X[k + 1][i] - X[0][i];
    // rows of J^{-1} (J has columns e_k): cofactors / det
    double cr[3][3];
    cr[0][0] = e[1][1] * e[2][2] - e[1][2] * e[2][1];
    cr[0][1] = e[1][2] * e[2][0] - e[1][0] * e[2][2];
    cr[0][2] = e[1][0] * e[2][1] - e[1][1] * e[2][0];
    cr[1][0] = e[2][1] * e[0][2] - e[2][2] * e[0][1];
    cr[1][1] = e[2][2] * e[0][0] - e[2][0] * e[0][2];
    cr[1][2] = e[2][0] * e[0][1] - e[2][1] * e[0][0];
    cr[2][0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
    cr[2][1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
    cr[2][2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
    const double det = e[0][0] * cr[0][0] + e[0][1] * cr[0][1] + e[0][2] * cr[0][2];
    const double idet = 1.0 / det;
    double gN[4][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gN[1][i] = cr[0][i] * idet;
        gN[2][i] = cr[1][i] * idet;
        gN[3][i] = cr[2][i] * idet;
        gN[0][i] = -(gN[1][i] + gN[2][i] + gN[3][i]);
    }
    const double w = det / 24.0;  // V/4
    // G = J^-T M J^-1, M = 2^{1/3}/2 [[2,1,1],[1,2,1],[1,1,2]]
    const double mc = 0.62996052494743658238;  // 2^{1/3} / 2
    double G[3][3];
    double GG = 0.0, trG = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int l = 0; l < 3; ++l) sum += gN[k + 1][i] * (k == l ? 2.0 : 1.0) * gN[l + 1][j];
            G[i][j] = mc * sum;
            GG += G[i][j] * G[i][j];
        }
    trG = G[0][0] + G[1][1] + G[2][2];

    double v[4][3], ac[4][3], p[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        p[c] = g.p[t[c]];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            v[c][i] = g.v[3 * (int64_t)t[c] + i];
            ac[c][i] = g.vdot[3 * (int64_t)t[c] + i];
        }
    }
    double gv[3][3], gp[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gp[i] = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) gv[i][j] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            gp[j] += p[c] * gN[c][j];
#pragma unroll
            for (int i = 0; i < 3; ++i) gv[i][j] += v[c][i] * gN[c][j];
        }
    const double div = gv[0][0] + gv[1][1] + gv[2][2];
    const double rho = g.rho, mu = g.mu, cm = g.c_m, cf = g.c_f;
    const double tconst = g.c_t / (g.dt * g.dt) + g.c_i * (mu / rho) * (mu / rho) * GG;

    // shape-function gradients of this lane's pair
    double ga[3], gb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ga[i] = pick(a, gN[0][i], gN[1][i], gN[2][i], gN[3][i]);
        gb[i] = pick(b, gN[0][i], gN[1][i], gN[2][i], gN[3][i]);
    }
    // viscous term of the residual of node a (constant per element)
    double visc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double sum = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) sum += ga[l] * (gv[i][l] + gv[l][i]);
        visc[i] = mu * sum;
    }
    const double gNab = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
    // (grad N_b . grad) v_i  = sum_l gN_b[l] gv[i][l]
    double gbv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) gbv[i] = gb[0] * gv[i][0] + gb[1] * gv[i][1] + gb[2] * gv[i][2];

    double A[3][3], B[3], C[3], D = 0.0, Rm[3], Rp = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        B[i] = 0.0;
        C[i] = 0.0;
        Rm[i] = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) A[i][j] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double vq[3], aq[3], pq = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            vq[i] = 0.0;
            aq[i] = 0.0;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double N = nq(q, c);
            pq += N * p[c];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                vq[i] += N * v[c][i];
                aq[i] += N * ac[c][i];
            }
        }
        double vGv = 0.0, conv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            conv[i] = gv[i][0] * vq[0] + gv[i][1] * vq[1] + gv[i][2] * vq[2];
#pragma unroll
            for (int j = 0; j < 3; ++j) vGv += vq[i] * G[i][j] * vq[j];
        }
        const double tM = (1.0 / rho) / sqrt(tconst + vGv);
        const double tC = 1.0 / (tM * trG);
        double vp[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) vp[i] = -tM * (rho * (aq[i] + conv[i]) + gp[i]);
        const double pp = -tC * div;
        double vpgv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) vpgv[i] = gv[i][0] * vp[0] + gv[i][1] * vp[1] + gv[i][2] * vp[2];

        const double Na = nq(q, a), Nb = nq(q, b);
        const double vgNa = vq[0] * ga[0] + vq[1] * ga[1] + vq[2] * ga[2];
        const double vgNb = vq[0] * gb[0] + vq[1] * gb[1] + vq[2] * gb[2];
        const double vpgNa = vp[0] * ga[0] + vp[1] * ga[1] + vp[2] * ga[2];
        const double vpgNb = vp[0] * gb[0] + vp[1] * gb[1] + vp[2] * gb[2];
        // residual of node a
#pragma unroll
        for (int i = 0; i < 3; ++i)
            Rm[i] += w * (rho * Na * (aq[i] + conv[i]) - ga[i] * pq + visc[i] - rho * vp[i] * vgNa +
                          rho * Na * vpgv[i] - rho * vp[i] * vpgNa - ga[i] * pp);
        Rp += w * (Na * div - vpgNa);

        // L_b (ij) = rho cm Nb d_ij + rho cf (d_ij v.gN_b + Nb d_j v_i): linearised rho(a + (v.grad)v)
        double L[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                L[i][j] = rho * cf * Nb * gv[i][j] + (i == j ? rho * (cm * Nb + cf * vgNb) : 0.0);
        // column sums used by the fine-scale terms
        double Lgv[3][3], LgNa[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            LgNa[j] = L[0][j] * ga[0] + L[1][j] * ga[1] + L[2][j] * ga[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) Lgv[i][j] = gv[i][0] * L[0][j] + gv[i][1] * L[1][j] + gv[i][2] * L[2][j];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double dij = (i == j) ? 1.0 : 0.0;
                double val = Na * L[i][j];                                   // rho N_a (a + (v.grad)v)
                val += mu * cf * (dij * gNab + ga[j] * gb[i]);               // 2 mu eps(w):eps(v)
                val += rho * tM * L[i][j] * vgNa - rho * cf * vp[i] * Nb * ga[j];  // -rho v'_i (v.gN_a)
                val += rho * Na * (-tM * Lgv[i][j] + cf * dij * vpgNb);      // rho N_a (v'.grad) v_i
                val += rho * tM * (L[i][j] * vpgNa + vp[i] * LgNa[j]);       // -rho v'_i (v'.gN_a)
                val += tC * cf * ga[i] * gb[j];                              // -d_i N_a p'
                A[i][j] += w * val;
            }
            B[i] += w * (-cf * ga[i] * Nb +
                         cf * rho * tM * (vgNa * gb[i] - Na * gbv[i] + gb[i] * vpgNa + vp[i] * gNab));
            C[i] += w * (cf * Na * gb[i] + tM * LgNa[i]);
        }
        D += w * cf * tM * gNab;
    }
    if (b == 0) {
        const int ta = a == 0 ? t[0] : a == 1 ? t[1] : a == 2 ? t[2] : t[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) g.res[3 * (int64_t)ta + i] += Rm[i];
        g.res[3 * (int64_t)g.N + ta] += Rp;
    }
    double* blk = g.aos + 16 * (int64_t)g.emap[16 * s + pair];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) blk[4 * i + j] += A[i][j];
        blk[4 * i + 3] += B[i];
        blk[12 + i] += C[i];
    }
    blk[15] += D;
}

void assemble_elements(const AsmArgs& a, hipStream_t st) {
    if (a.count <= 0) return;
    hipLaunchKernelGGL(k_assemble_elements, dim3(grid_for((int64_t)kPairs * a.count)), dim3(kBlock), 0, st, a);
}

// Backflow term -rho beta (v.n)_- N_a v_i on outlet triangles (3-point rule,
// (x)_- derivative 1 for x < 0 and 0 otherwise).
__global__ void k_assemble_faces(FaceArgs g) {
    const int s = g.F0 + blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.F0 + g.count) return;
    int nd[3];
    double X[3][3], v[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nd[a] = g.faces[3 * (int64_t)s + a];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            X[a][i] = g.xyz[3 * (int64_t)nd[a] + i];
            v[a][i] = g.v[3 * (int64_t)nd[a] + i];
        }
    }
    double e1[3], e2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        e1[i] = X[1][i] - X[0][i];
        e2[i] = X[2][i] - X[0][i];
    }
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double area = 0.5 * len;
#pragma unroll
    for (int i = 0; i < 3; ++i) n[i] /= len;
    const double w = area / 3.0;
    const double k0 = -g.rho * g.beta;
    double R[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double A[3][3][3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) A[a][b][i][j] = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double N[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) N[a] = (a == q) ? (2.0 / 3.0) : (1.0 / 6.0);
        double vq[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) vq[i] = N[0] * v[0][i] + N[1] * v[1][i] + N[2] * v[2][i];
        const double vn = vq[0] * n[0] + vq[1] * n[1] + vq[2] * n[2];
        const double neg = vn < 0.0 ? vn : 0.0;
        const double H = vn < 0.0 ? 1.0 : 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int i = 0; i < 3; ++i) R[a][i] += w * k0 * neg * N[a] * vq[i];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        A[a][b][i][j] +=
                            w * k0 * g.c_f * (H * N[b] * n[j] * N[a] * vq[i] + (i == j ? neg * N[a] * N[b] : 0.0));
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int i = 0; i < 3; ++i) g.res[3 * (int64_t)nd[a] + i] += R[a][i];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double* blk = g.aos + 16 * (int64_t)g.fmap[9 * (int64_t)s + 3 * a + b];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) blk[4 * i + j] += A[a][b][i][j];
        }
    }
}

void assemble_faces(const FaceArgs& a, hipStream_t st) {
    if (a.count <= 0) return;
    hipLaunchKernelGGL(k_assemble_faces, dim3(grid_for(a.count)), dim3(kBlock), 0, st, a);
}

// a^k_{A i} += (|f|/3) n_i for the nodes of each outlet face (colour by colour)
__global__ void k_outlet_vectors(int F0, int count, const int32_t* faces, const int32_t* fslot, const double* xyz,
                                 double* a_raw) {
    const int s = F0 + blockIdx.x * kBlock + threadIdx.x;
    if (s >= F0 + count) return;
    double X[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) X[a][i] = xyz[3 * (int64_t)faces[3 * (int64_t)s + a] + i];
    double e1[3], e2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        e1[i] = X[1][i] - X[0][i];
        e2[i] = X[2][i] - X[0][i];
    }
    // |f|/3 n = cross / 6
    const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t sl = fslot[3 * (int64_t)s + a];
#pragma unroll
        for (int i = 0; i < 3; ++i) a_raw[3 * sl + i] += c[i] / 6.0;
    }
}
void outlet_vectors(int F0, int count, const int32_t* faces, const int32_t* fslot, const double* xyz, double* a_raw,
                    hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_outlet_vectors, dim3(grid_for(count)), dim3(kBlock), 0, st, F0, count, faces, fslot, xyz,
                       a_raw);
}

__global__ void k_mask_outlet(int n_slots, const int32_t* onode, const uint8_t* mask, const double* a_raw,
                              double* a_msk) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n_slots * 3) return;
    const int sl = (int)(t / 3), c = (int)(t % 3);
    a_msk[t] = mask[4 * (int64_t)onode[sl] + c] ? 0.0 : a_raw[t];
}
void mask_outlet(int n_slots, const int32_t* onode, const uint8_t* mask, const double* a_raw, double* a_msk,
                 hipStream_t st) {
    if (n_slots <= 0) return;
    hipLaunchKernelGGL(k_mask_outlet, dim3(grid_for((int64_t)n_slots * 3)), dim3(kBlock), 0, st, n_slots, onode,
                       mask, a_raw, a_msk);
}

// [nnzb][16] -> [16][nnzb] with Dirichlet rows/columns replaced by the identity
__global__ void k_finalize_tangent(int64_t nnzb, const int32_t* row_of, const int32_t* col, const uint8_t* mask,
                                   const double* aos, double* V) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nnzb) return;
    const int i = row_of[k], j = col[k];
    const uchar4 mi = *reinterpret_cast<const uchar4*>(mask + 4 * (int64_t)i);
    const uchar4 mj = *reinterpret_cast<const uchar4*>(mask + 4 * (int64_t)j);
    const uint8_t ri[4] = {mi.x, mi.y, mi.z, mi.w};
    const uint8_t cj[4] = {mj.x, mj.y, mj.z, mj.w};
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double val = aos[16 * k + 4 * r + c];
            if (ri[r] || cj[c]) val = (i == j && r == c) ? 1.0 : 0.0;
            V[(4 * r + c) * nnzb + k] = val;
        }
}
void finalize_tangent(int64_t nnzb, const int32_t* row_of, const int32_t* col, const uint8_t* mask,
                      const double* aos, double* V, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_tangent, dim3(grid_for(nnzb)), dim3(kBlock), 0, st, nnzb, row_of, col, mask, aos,
                       V);
}

__global__ void k_finalize_rhs(int N, const uint8_t* mask, const double* res, double* rhs) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 4 * (int64_t)N) return;
    const int64_t node = t < 3 * (int64_t)N ? t / 3 : t - 3 * (int64_t)N;
    const int c = t < 3 * (int64_t)N ? (int)(t % 3) : 3;
    rhs[t] = mask[4 * node + c] ? 0.0 : -res[t];
}
void finalize_rhs(int N, const uint8_t* mask, const double* res, double* rhs, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_rhs, dim3(grid_for(4 * (int64_t)N)), dim3(kBlock), 0, st, N, mask, res, rhs);
}

__global__ void k_add_traction(int n_slots, const int32_t* onode, const int32_t* oid, const double* P_af,
                               const double* a_raw, double* res) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n_slots * 3) return;
    const int sl = (int)(t / 3), c = (int)(t % 3);
    res[3 * (int64_t)onode[sl] + c] += P_af[oid[sl]] * a_raw[t];
}
void add_traction(int n_slots, const int32_t* onode, const int32_t* oid, const double* P_af, const double* a_raw,
                  double* res, hipStream_t st) {
    if (n_slots <= 0) return;
    hipLaunchKernelGGL(k_add_traction, dim3(grid_for((int64_t)n_slots * 3)), dim3(kBlock), 0, st, n_slots, onode,
                       oid, P_af, a_raw, res);
}

// Resistance outlets (Sec. 2.5): m^k = R^k enters the rank-one weight
// c_k = c_f R^k, and the traction pressure is
// P^k_{n+af} = (1 - alpha_f) P^k_n + alpha_f R^k Q^k (P_n == nullptr: P_n = R Q).
__global__ void k_resistance_outlets(int n_out, const double* R, const double* P_n, const double* Q, double af,
                                     double cf, double* ck, double* P_af) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_out) return;
    const double rq = R[k] * Q[k];
    ck[k] = cf * R[k];
    P_af[k] = (1.0 - af) * (P_n ? P_n[k] : rq) + af * rq;
}
void resistance_outlets(int n_out, const double* R, const double* P_n, const double* Q, double af, double cf,
                        double* ck, double* P_af, hipStream_t st) {
    if (n_out <= 0) return;
    hipLaunchKernelGGL(k_resistance_outlets, dim3(grid_for(n_out)), dim3(kBlock), 0, st, n_out, R, P_n, Q, af, cf,
                       ck, P_af);
}

// dL/dR_k = lambda^T (dr/dR_k - (dA/dR_k) x) with dr/dR_k = -[alpha_f Q^k a^k; 0]
// and dA/dR_k = blockdiag(c_f a^k a^k^T, 0): -(a^k.lambda_v)(alpha_f Q^k + c_f a^k.x_v),
// from the masked dots s_lam[k] = a^k.lambda_v and s_x[k] = a^k.x_v.
__global__ void k_resistance_grad(int n_out, const double* s_lam, const double* s_x, const double* Q, double af,
                                  double cf, double* grad) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_out) return;
    grad[k] = -s_lam[k] * (af * Q[k] + cf * s_x[k]);
}
void resistance_grad(int n_out, const double* s_lam, const double* s_x, const double* Q, double af, double cf,
                     double* grad, hipStream_t st) {
    if (n_out <= 0) return;
    hipLaunchKernelGGL(k_resistance_grad, dim3(grid_for(n_out)), dim3(kBlock), 0, st, n_out, s_lam, s_x, Q, af, cf,
                       grad);
}

}  // namespace ns
