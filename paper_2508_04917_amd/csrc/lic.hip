// Learned interface correction (an addition to the paper's method; the paper
// has no learned component).
//
// Faces are the directed cut pairs (I, J): the blocks A_IJ of the full
// reordered matrix whose row and column lie in different subdomains (the
// blocks the drop removes), in CSR order.  A per-face MLP 27 -> 64 -> 64 -> 9
// (FP32) maps x_f = [A_II, A_IJ, A_JJ] / sigma_f, sigma_f =
// sqrt(|tr A_II| |tr A_JJ|) / 3, to a 3x3 coefficient C_f, and the
// preconditioner becomes z = M_DD^{-1} (r + C r), (C r)_I = sum_f C_f r_J:
// a fixed linear operator once C is set, so BiCGSTAB stays valid.  The
// correction is applied inside the apply kernel right after the subdomain's
// r is staged in LDS (it reads only r).
//
// Training regresses the corrected apply onto the global ILU0 apply on probe
// vectors: loss = mean_q ||z_q - z*_q||^2 / ||z_DD,q - z*_q||^2; its
// gradient is dL/dC_f = sum_q a_q[I] r_q[J]^T with a_q = M_DD^{-T} g_q,
// g_q = 2 (z_q - z*_q) / (Q den_q), computed with the same apply kernel run
// on the transposed factors, then backpropagated through the MLP.
#include "internal.h"

namespace ddilu {

constexpr int kIn = 27, kHid = 64, kOut = 9;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid, kNParam = oB3 + kOut;
static_assert(kNParam == 6537, "parameter count");

// ------------------------------------------------------------------ faces
__global__ void k_face_count(int64_t n, int S, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                             int32_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = i / S;
    int c = 0;
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q) c += (col[q] / S != s);
    cnt[i] = c;
}

__global__ void k_face_fill(int64_t n, int S, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ fptr, int32_t *fI, int32_t *fJ, int32_t *fq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = i / S;
    int32_t f = fptr[i];
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q)
        if (col[q] / S != s) {
            fI[f] = (int32_t)i;
            fJ[f] = col[q];
            fq[f] = q;
            ++f;
        }
}

// Rank-major faces (the apply's copy): faces of rank k (a row's k-th face)
// of subdomain s occupy positions fptr[sS] + rb[9s + k] ... in row order.
// One pass per rank present: flag the rows with more than k faces, scan, and
// place their k-th faces; rb[9s + k + 1] = rb[9s + k] + rows of s flagged.
__global__ void k_rank_flag(int64_t n, int k, const int32_t *__restrict__ fptr, int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = fptr[i + 1] - fptr[i] > k;
}

__global__ void k_rank_place(int64_t n, int S, int k, const int32_t *__restrict__ fptr, const int32_t *__restrict__ fJ,
                             const int32_t *__restrict__ pre, const int32_t *__restrict__ rb, int2 *lrec,
                             int32_t *lperm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || fptr[i + 1] - fptr[i] <= k) return;
    const int64_t s = i / S, b = s * S;
    const int32_t pos = fptr[b] + rb[9 * s + k] + (pre[i] - pre[b]);
    const int32_t f = fptr[i] + k;
    lrec[pos] = make_int2((int32_t)(i - b), fJ[f]);
    lperm[pos] = f;
}

__global__ void k_rank_count(int nsub, int S, int k, const int32_t *__restrict__ pre, int32_t *rb) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsub) rb[9 * s + k + 1] = rb[9 * s + k] + (pre[(int64_t)(s + 1) * S] - pre[(int64_t)s * S]);
}

// the apply's copy of C: Cr[p] = C[lperm[p]]
__global__ void k_rank_coeffs(int64_t nf, const int32_t *__restrict__ lperm, const float *__restrict__ C, float *Cr) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nf * 9) return;
    const int64_t p = e / 9;
    Cr[e] = C[(int64_t)lperm[p] * 9 + (e - p * 9)];
}

// status[7] = the most faces of any row (the apply's rank table holds 8);
// a maximum over the workgroup first, then one atomic per workgroup
__global__ __launch_bounds__(256) void k_face_limits(int64_t n, const int32_t *__restrict__ fptr, int32_t *status) {
    __shared__ int32_t wmax[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t m = i < n ? fptr[i + 1] - fptr[i] : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, __shfl_xor(m, d));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = max(m, wmax[w]);
        if (m > 0) atomicMax(&status[7], m);
    }
}

__global__ void k_sym_check(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            int32_t *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q) {
        const int32_t j = col[q];
        bool found = false;
        for (int32_t r = ptr[j]; r < ptr[j + 1]; ++r) found |= (col[r] == i);
        if (!found) atomicMax(&status[6], 1);
    }
}

__global__ void k_features(int64_t nf, const int32_t *__restrict__ fI, const int32_t *__restrict__ fJ,
                           const int32_t *__restrict__ fq, const int32_t *__restrict__ diag,
                           const double *__restrict__ val, float *X) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const double *Aii = val + (int64_t)diag[fI[f]] * 9, *Aij = val + (int64_t)fq[f] * 9;
    const double *Ajj = val + (int64_t)diag[fJ[f]] * 9;
    const double ti = Aii[0] + Aii[4] + Aii[8], tj = Ajj[0] + Ajj[4] + Ajj[8];
    const double sigma = sqrt(fabs(ti) * fabs(tj)) / 3.0;
    float *x = X + f * kIn;
    for (int e = 0; e < 9; ++e) {
        x[e] = (float)(Aii[e] / sigma);
        x[9 + e] = (float)(Aij[e] / sigma);
        x[18 + e] = (float)(Ajj[e] / sigma);
    }
}

// ---------------------------------------------------------------- MLP (FP32)
// On the matrix cores (v_mfma_f32_16x16x4_f32: D[16][16] += A[16][4] B[4][16];
// lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds
// D[4(l/16) + r][l%16] in accumulator r).  A wavefront evaluates 16 faces at
// a time with the faces along the columns.  Layer 1 is H1^T (64 x 16) =
// W1 (64 x 27) X^T as four 16-row tiles over seven steps of four inputs (the
// 28th input a zero), so lane l = 16 g + j ends with H1^T[16 t + 4 g + r]
// [face j] in accumulator r of tile t.  Layers 2 and 3 take those registers
// as their B operand unchanged by visiting their 64 inputs in the order the
// layout gives (step (t', r) takes inputs 16 t' + 4 g + r from lane group g;
// every input once), with the weight operand loaded in that same order.
// The weight operands stay in registers for all of a wavefront's faces.
typedef float mf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf4 mfma4(float a, float b, mf4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kMlpBlocks = 2048;  // workgroups of 4 wavefronts, each looping over tiles of 16 faces

// C = W3 relu(W2 relu(W1 x + b1) + b2) + b3 per face; with H1/H2 given the
// hidden activations are kept for the backward pass.
__global__ __launch_bounds__(256) void k_mlp_forward(int64_t nf, const float *__restrict__ P,
                                                     const float *__restrict__ X, float *__restrict__ C,
                                                     float *__restrict__ H1, float *__restrict__ H2) {
    const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
    float w1[4][7], w2[4][16], w3[16], b1[4][4], b2[4][4], b3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            const int k = 4 * s + g;
            w1[t][s] = k < kIn ? P[oW1 + (16 * t + j) * kIn + k] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) w2[t][u] = P[oW2 + (16 * t + j) * kHid + 16 * (u >> 2) + 4 * g + (u & 3)];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            b1[t][r] = P[oB1 + 16 * t + 4 * g + r];
            b2[t][r] = P[oB2 + 16 * t + 4 * g + r];
        }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) w3[u] = j < kOut ? P[oW3 + j * kHid + 16 * (u >> 2) + 4 * g + (u & 3)] : 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) b3[r] = 4 * g + r < kOut ? P[oB3 + 4 * g + r] : 0.f;

    // one wavefront per SIMD fits these registers: the next tile's inputs are
    // fetched while the current tile computes
    auto fetch_x = [&](int64_t tile, float (&xb)[7]) {
        const int64_t f = tile * 16 + j;
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            const int k = 4 * s + g;
            xb[s] = (f < nf && k < kIn) ? X[f * kIn + k] : 0.f;
        }
    };
    const int64_t ntile = (nf + 15) / 16, tstep = (int64_t)gridDim.x * 4;
    float xn[7];
    fetch_x((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), xn);
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntile; tile += tstep) {
        const int64_t f = tile * 16 + j;
        const bool fok = f < nf;
        float xb[7];
#pragma unroll
        for (int s = 0; s < 7; ++s) xb[s] = xn[s];
        fetch_x(tile + tstep, xn);
        mf4 h1[4], h2[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            mf4 acc = {b1[t][0], b1[t][1], b1[t][2], b1[t][3]};
#pragma unroll
            for (int s = 0; s < 7; ++s) acc = mfma4(w1[t][s], xb[s], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = acc[r] > 0.f ? acc[r] : 0.f;
            h1[t] = acc;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            mf4 acc = {b2[t][0], b2[t][1], b2[t][2], b2[t][3]};
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = mfma4(w2[t][u], h1[u >> 2][u & 3], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = acc[r] > 0.f ? acc[r] : 0.f;
            h2[t] = acc;
        }
        mf4 o = {b3[0], b3[1], b3[2], b3[3]};
#pragma unroll
        for (int u = 0; u < 16; ++u) o = mfma4(w3[u], h2[u >> 2][u & 3], o);
        if (fok) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (4 * g + r < kOut) C[f * kOut + 4 * g + r] = o[r];
            if (H1) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    *reinterpret_cast<mf4 *>(H1 + f * kHid + 16 * t + 4 * g) = h1[t];
                    *reinterpret_cast<mf4 *>(H2 + f * kHid + 16 * t + 4 * g) = h2[t];
                }
            }
        }
    }
}

// Backward through the two hidden layers, per face: G2 = W3^T dOUT (masked by
// h2 > 0), G1 = W2^T G2 (masked by h1 > 0); the same tiling as the forward
// pass, the transposed weights as the A operand.
__global__ __launch_bounds__(256) void k_mlp_backprop(int64_t nf, const float *__restrict__ P,
                                                      const float *__restrict__ dOUT, const float *__restrict__ H1,
                                                      const float *__restrict__ H2, float *__restrict__ G1,
                                                      float *__restrict__ G2) {
    const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
    float w3t[4][3], w2t[4][16];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int k = 4 * s + g;
            w3t[t][s] = k < kOut ? P[oW3 + k * kHid + 16 * t + j] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) w2t[t][u] = P[oW2 + (16 * (u >> 2) + 4 * g + (u & 3)) * kHid + 16 * t + j];
    }
    const int64_t ntile = (nf + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntile; tile += (int64_t)gridDim.x * 4) {
        const int64_t f = tile * 16 + j;
        const bool fok = f < nf;
        const int64_t fc = fok ? f : 0;  // a valid face for the masks' loads
        float db[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int k = 4 * s + g;
            db[s] = (fok && k < kOut) ? dOUT[f * kOut + k] : 0.f;
        }
        mf4 g2[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            mf4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 3; ++s) acc = mfma4(w3t[t][s], db[s], acc);
            const mf4 h = *reinterpret_cast<const mf4 *>(H2 + fc * kHid + 16 * t + 4 * g);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = h[r] > 0.f ? acc[r] : 0.f;
            g2[t] = acc;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            mf4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = mfma4(w2t[t][u], g2[u >> 2][u & 3], acc);
            const mf4 h = *reinterpret_cast<const mf4 *>(H1 + fc * kHid + 16 * t + 4 * g);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = h[r] > 0.f ? acc[r] : 0.f;
            if (fok) {
                *reinterpret_cast<mf4 *>(G1 + f * kHid + 16 * t + 4 * g) = acc;
                *reinterpret_cast<mf4 *>(G2 + f * kHid + 16 * t + 4 * g) = g2[t];
            }
        }
    }
}

static unsigned mlp_blocks(int64_t nf) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(((nf + 15) / 16 + 3) / 4, kMlpBlocks));
}

// Weight gradients on the matrix cores.  Layer l's gradient is a product
// over faces, dW[i][k] = sum_f A[f][i] B[f][k] with A = dOUT / G2 / G1 and
// B = H2 / H1 / X, and its bias gradient db[i] = sum_f A[f][i] is the same
// product with a column of ones appended to B.  The outputs are cut into
// 16x16 tiles (layer 0: 1 x 5 tiles of 9 x 65 entries, layer 1: 4 x 5 of
// 64 x 65, layer 2: 4 x 2 of 64 x 28; 33 tiles, every parameter in exactly
// one), and one wavefront accumulates one tile over one chunk of kWgFaces
// faces with v_mfma_f32_16x16x4_f32 (four faces per instruction: lane l
// supplies A[f0 + l/16][i0 + l%16] and B[f0 + l/16][k0 + l%16], and holds
// D[i0 + 4(l/16) + r][k0 + l%16] in accumulator r).  Positions outside a
// layer's matrix contribute zeros.  The chunk's tile is written as FP64
// partials and k_wgrad_sum adds the chunks in order, so the result does not
// depend on timing.
constexpr int kWgFaces = 256;  // faces per chunk
constexpr int kWgTiles = 33;   // 16x16 output tiles over the three layers

__global__ __launch_bounds__(256) void k_wgrad_mfma(int64_t nf, const float *__restrict__ dOUT,
                                                    const float *__restrict__ G2, const float *__restrict__ G1,
                                                    const float *__restrict__ H2, const float *__restrict__ H1,
                                                    const float *__restrict__ X, double *__restrict__ part) {
    const int chunk = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (tile >= kWgTiles) return;  // whole wavefronts
    const float *A, *B;
    int na, nb, ow, ob, ti, tk;
    if (tile < 5) {
        A = dOUT; na = kOut; B = H2; nb = kHid; ow = oW3; ob = oB3; ti = 0; tk = tile;
    } else if (tile < 25) {
        A = G2; na = kHid; B = H1; nb = kHid; ow = oW2; ob = oB2; ti = (tile - 5) / 5; tk = (tile - 5) % 5;
    } else {
        A = G1; na = kHid; B = X; nb = kIn; ow = oW1; ob = oB1; ti = (tile - 25) / 2; tk = (tile - 25) % 2;
    }
    const int i = ti * 16 + (lane & 15), k = tk * 16 + (lane & 15), fl = lane >> 4;
    const int64_t f0 = (int64_t)chunk * kWgFaces;
    mf4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
    for (int g = 0; g < kWgFaces; g += 4) {
        const int64_t f = f0 + g + fl;
        const bool fok = f < nf;
        const float a = (fok && i < na) ? A[f * na + i] : 0.f;
        const float b = !fok ? 0.f : (k < nb ? B[f * nb + k] : (k == nb ? 1.f : 0.f));
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    double *out = part + (int64_t)chunk * kNParam;
    const int col = tk * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = ti * 16 + 4 * (lane >> 4) + r;
        if (row < na) {
            if (col < nb) out[ow + row * nb + col] = (double)acc[r];
            else if (col == nb) out[ob + row] = (double)acc[r];
        }
    }
}

__global__ void k_wgrad_sum(int nchunk, const double *__restrict__ part, float *grad, int accumulate) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNParam) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * kNParam + e];
    grad[e] = accumulate ? grad[e] + (float)s : (float)s;
}

// ----------------------------------------------------------- training steps
// g = 2 (z - z*) / (Q den_q) for probe q (grid.y), and per-workgroup partial
// sums of ||z - z*||^2.
__global__ __launch_bounds__(256) void k_lic_residual(int64_t m, const double *__restrict__ z,
                                                      const double *__restrict__ zs, const double *__restrict__ den,
                                                      int Q, double *__restrict__ g, double *__restrict__ part,
                                                      int part_stride) {
    const int q = blockIdx.y;
    const double sc = 2.0 / (Q * den[q]);
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const double e = z[q * m + i] - zs[q * m + i];
        g[q * m + i] = sc * e;
        acc += e * e;
    }
    __shared__ double sh[4];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
        part[q * part_stride + blockIdx.x] = t;
    }
}

// loss += sum_q (sum of partials of probe q) / (Q den_q); one workgroup.
// Thread t adds partials t, t + kLossT, ... of each probe in order, then a
// fixed tree over the workgroup, probes in order: the result does not depend
// on timing.
constexpr int kLossT = 256;

__global__ __launch_bounds__(kLossT) void k_lic_loss(int Q, int nblk, int part_stride,
                                                     const double *__restrict__ part,
                                                     const double *__restrict__ den, double *loss) {
    __shared__ double sh[kLossT];
    double L = 0.0;
    for (int q = 0; q < Q; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kLossT) s += part[q * part_stride + b];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = kLossT / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) L += sh[0] / (Q * den[q]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss += L;
}

// den_q = ||z_DD,q - z*_q||^2 (one workgroup per probe, fixed order).
__global__ __launch_bounds__(256) void k_lic_den(int64_t m, const double *__restrict__ zdd,
                                                 const double *__restrict__ zs, double *den) {
    const int q = blockIdx.x;
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
        const double e = zdd[q * m + i] - zs[q * m + i];
        acc += e * e;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) den[q] = sh[0];
}

// dC_f[a][b] = sum_q a_q[I][a] r_q[J][b] (FP32 result, FP64 sum).
__global__ void k_lic_dC(int64_t nf, int64_t m, int Q, const int32_t *__restrict__ fI, const int32_t *__restrict__ fJ,
                         const double *__restrict__ A, const double *__restrict__ R, float *dC) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nf * 9) return;
    const int64_t f = t / 9;
    const int a = (int)(t % 9) / 3, b = (int)(t % 3);
    const int64_t I = fI[f], J = fJ[f];
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s += A[q * m + I * 3 + a] * R[q * m + J * 3 + b];
    dC[t] = (float)s;
}

// Adam (Kingma & Ba) on FP32 parameters.
__global__ void k_adam(int np, float *P, const float *__restrict__ G, float *M, float *V, float c1, float c2, float lr,
                       float b1, float b2, float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float g = G[i];
    const float m = b1 * M[i] + (1.f - b1) * g;
    const float v = b2 * V[i] + (1.f - b2) * g * g;
    M[i] = m;
    V[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ------------------------------------------------------------ adjoint streams
// Values of the transposed sweeps in the slot layout (same positions and
// columns as the forward sweeps, which requires a structurally symmetric
// pattern; lane-contiguous runs as in the forward streams): lower sweep of
// U^T: slot k of row I holds (Uhat_{J_k I})^T; upper sweep of L^T: slot k
// holds (L_{K_k I})^T, followed by inv_D_I^T.
__global__ void k_pack_adjoint(int64_t n, int S, int which, int MB, const int32_t *__restrict__ tptr,
                               const int32_t *__restrict__ tcol, const double *__restrict__ lu,
                               const double *__restrict__ invd, const int32_t *__restrict__ rows, double *sval) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t base = (p / S) * (int64_t)S;
    const int64_t gi = base + rows[p];
    const int NV = (MB + which) * 3;
    double *o = sval + p * 3 * NV;
    int k = 0;
    for (int32_t q = tptr[gi]; q < tptr[gi + 1] && k < MB; ++q) {
        const int32_t c = tcol[q];
        if (which == 0 ? (c < gi) : (c > gi)) {
            int32_t qt = -1;  // position of (c, gi) in row c (exists: symmetric pattern)
            for (int32_t r = tptr[c]; r < tptr[c + 1]; ++r)
                if (tcol[r] == gi) qt = r;
            double blk[9];
            if (qt < 0) {
                for (int e = 0; e < 9; ++e) blk[e] = 0.0;
            } else if (which == 0) {  // Uhat_{c,gi} = inv_D_c U_{c,gi}
                const double *a = invd + (int64_t)c * 9, *b = lu + (int64_t)qt * 9;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double s = 0.0;
                        for (int l = 0; l < 3; ++l) s += a[i * 3 + l] * b[l * 3 + j];
                        blk[i * 3 + j] = s;
                    }
            } else {  // L_{c,gi}
                for (int e = 0; e < 9; ++e) blk[e] = lu[(int64_t)qt * 9 + e];
            }
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) o[i * NV + k * 3 + j] = blk[j * 3 + i];
            ++k;
        }
    }
    for (; k < MB; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) o[i * NV + k * 3 + j] = 0.0;
    if (which == 1) {
        const double *a = invd + gi * 9;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) o[i * NV + MB * 3 + j] = a[j * 3 + i];
    }
}

// ------------------------------------------------------------------ setup
int lic_setup(dd_ctx *h, hipStream_t st) {
    if (h->bs != 3) return h->fail(DD_EINVAL, "the learned correction needs 3x3 blocks");
    if (!h->factored) return h->fail(DD_ESTATE, "lic_setup before ilu0_factor");
    if (h->slots == 0) return h->fail(DD_EINVAL, "the learned correction needs the slot layout (rows of <= 3 blocks)");
    const int T = 256;
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    Lic &L = h->lic;
    hipError_t e;
    const int32_t st67[2] = {0, 0};
    e = hipMemcpyAsync(h->status + 6, st67, 2 * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "memcpy: %s", hipGetErrorString(e));
    k_sym_check<<<g, T, 0, st>>>(h->n, h->aptr, h->acol, h->status);
    int32_t *cnt = nullptr, *flag = nullptr, *bpos = nullptr;
    int rc = h->alloc(&cnt, h->n);
    if (!rc) rc = h->alloc(&flag, h->n);
    if (!rc) rc = h->alloc(&bpos, h->n + 1);
    if (!rc && !L.fptr) rc = h->alloc(&L.fptr, h->n + 1);
    if (!rc && !L.diag) rc = h->alloc(&L.diag, h->n);
    if (!rc && !L.rb) rc = h->alloc(&L.rb, 9 * (int64_t)h->nsub);
    if (rc) return rc;
    k_face_count<<<g, T, 0, st>>>(h->n, h->S, h->aptr, h->acol, cnt);
    e = exclusive_scan(cnt, L.fptr, h->n, h->scan_tmp, st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "scan: %s", hipGetErrorString(e));
    k_face_limits<<<g, T, 0, st>>>(h->n, L.fptr, h->status);
    int32_t nf = 0, sym[2] = {0, 0};
    e = hipMemcpyAsync(&nf, L.fptr + h->n, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sym, h->status + 6, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic setup: %s", hipGetErrorString(e));
    if (sym[0]) return h->fail(DD_EINVAL, "the learned correction needs a structurally symmetric pattern");
    const int maxrank = sym[1];
    if (maxrank > 8) return h->fail(DD_EINVAL, "the learned correction supports at most 8 cut faces per row");
    L.nf = nf;
    for (void *q : {(void *)L.fI, (void *)L.fJ, (void *)L.fq, (void *)L.X, (void *)L.C, (void *)L.lrec,
                    (void *)L.lperm, (void *)L.Cr})
        if (q) {
            h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), q));
            (void)hipFree(q);
        }
    rc = h->alloc(&L.fI, nf);
    if (!rc) rc = h->alloc(&L.fJ, nf);
    if (!rc) rc = h->alloc(&L.fq, nf);
    if (!rc) rc = h->alloc(&L.X, (int64_t)nf * kIn);
    if (!rc) rc = h->alloc(&L.C, (int64_t)nf * kOut);
    if (!rc) rc = h->alloc(&L.lrec, nf);
    if (!rc) rc = h->alloc(&L.lperm, nf);
    if (!rc) rc = h->alloc(&L.Cr, (int64_t)nf * kOut);
    if (rc) return rc;
    k_face_fill<<<g, T, 0, st>>>(h->n, h->S, h->aptr, h->acol, L.fptr, L.fI, L.fJ, L.fq);
    // the apply's rank-major copy of the faces
    e = hipMemsetAsync(L.rb, 0, 9 * (size_t)h->nsub * sizeof(int32_t), st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "memset: %s", hipGetErrorString(e));
    const unsigned gs = (unsigned)((h->nsub + T - 1) / T);
    for (int k = 0; k < 8; ++k) {
        if (k < maxrank) {
            k_rank_flag<<<g, T, 0, st>>>(h->n, k, L.fptr, flag);
            e = exclusive_scan(flag, bpos, h->n, h->scan_tmp, st);
            if (e != hipSuccess) return h->fail(DD_EHIP, "scan: %s", hipGetErrorString(e));
            k_rank_place<<<g, T, 0, st>>>(h->n, h->S, k, L.fptr, L.fJ, bpos, L.rb, L.lrec, L.lperm);
        } else {
            // no row has more than k faces: the boundaries after the last rank repeat
            e = hipMemsetAsync(bpos, 0, (h->n + 1) * sizeof(int32_t), st);
            if (e != hipSuccess) return h->fail(DD_EHIP, "memset: %s", hipGetErrorString(e));
        }
        k_rank_count<<<gs, T, 0, st>>>(h->nsub, h->S, k, bpos, L.rb);
    }
    hipError_t ed = launch_diag_positions(h, L.diag, st);
    if (ed != hipSuccess) return h->fail(DD_EHIP, "diag: %s", hipGetErrorString(ed));
    if (nf) k_features<<<(unsigned)((nf + T - 1) / T), T, 0, st>>>(nf, L.fI, L.fJ, L.fq, L.diag, h->aval, L.X);
    // the adjoint apply's streams are packed on first use (training only)
    L.adj_ready = 0;
    e = hipStreamSynchronize(st);
    for (void *q : {(void *)cnt, (void *)flag, (void *)bpos}) {
        h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), q));
        (void)hipFree(q);
    }
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic setup: %s", hipGetErrorString(e));
    L.ready = 1;
    L.active = 0;
    return DD_OK;
}

int lic_adjoint_streams(dd_ctx *h, hipStream_t st) {
    Lic &L = h->lic;
    if (!L.ready) return h->fail(DD_ESTATE, "the adjoint apply needs lic_setup");
    if (L.adj_ready) return DD_OK;
    const int T = 256, bb = 9;
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    for (int w = 0; w < 2; ++w) {
        if (!L.adj_val[w]) {
            int rc = h->alloc(&L.adj_val[w], h->n * (h->slots + w) * bb);
            if (rc) return rc;
        }
    }
    for (int w = 0; w < 2; ++w)
        k_pack_adjoint<<<g, T, 0, st>>>(h->n, h->S, w, h->slots, h->tptr, h->tcol, h->lu, h->invd,
                                        h->lev[w].rows, L.adj_val[w]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return h->fail(DD_EHIP, "adjoint streams: %s", hipGetErrorString(e));
    L.adj_ready = 1;
    return DD_OK;
}

// The apply reads the coefficients in rank-major order: refresh that copy
// after every change of C.
int lic_publish_coeffs(dd_ctx *h, hipStream_t st) {
    Lic &L = h->lic;
    if (L.nf) k_rank_coeffs<<<(unsigned)(((int64_t)L.nf * 9 + 255) / 256), 256, 0, st>>>(L.nf, L.lperm, L.C, L.Cr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return h->fail(DD_EHIP, "coefficients: %s", hipGetErrorString(e));
    return DD_OK;
}

int lic_coeffs_from_params(dd_ctx *h, const float *params, bool keep_hidden, hipStream_t st) {
    Lic &L = h->lic;
    if (keep_hidden && !L.H1) {
        int rc = h->alloc(&L.H1, (int64_t)std::max(L.nf, 1) * kHid);
        if (!rc) rc = h->alloc(&L.H2, (int64_t)std::max(L.nf, 1) * kHid);
        if (rc) return rc;
    }
    if (L.nf)
        k_mlp_forward<<<mlp_blocks(L.nf), 256, 0, st>>>(L.nf, params, L.X, L.C, keep_hidden ? L.H1 : nullptr,
                                                        keep_hidden ? L.H2 : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return h->fail(DD_EHIP, "mlp forward: %s", hipGetErrorString(e));
    return lic_publish_coeffs(h, st);
}

// Loss and gradient of one problem (see the file comment); adds to *loss and
// (accumulate != 0) to grad.
int lic_loss_grad_run(dd_ctx *h, const float *params, int Q, const double *R, const double *Zs, const double *den,
                      double *loss, float *grad, int accumulate, hipStream_t st) {
    Lic &L = h->lic;
    const int64_t m = h->n * 3;
    int rc = lic_coeffs_from_params(h, params, true, st);
    if (rc) return rc;
    if (L.work_q < Q) {
        for (void *q : {(void *)L.Z, (void *)L.G, (void *)L.A, (void *)L.rpart})
            if (q) {
                h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), q));
                (void)hipFree(q);
            }
        rc = h->alloc(&L.Z, Q * m);
        if (!rc) rc = h->alloc(&L.G, Q * m);
        if (!rc) rc = h->alloc(&L.A, Q * m);
        if (!rc) rc = h->alloc(&L.rpart, (int64_t)Q * 2048);
        if (rc) return rc;
        L.work_q = Q;
    }
    if (!L.dC) {
        rc = h->alloc(&L.dC, (int64_t)std::max(L.nf, 1) * 9);
        if (!rc) rc = h->alloc(&L.G1, (int64_t)std::max(L.nf, 1) * kHid);
        if (!rc) rc = h->alloc(&L.G2, (int64_t)std::max(L.nf, 1) * kHid);
        const int nchunk = (int)((std::max(L.nf, 1) + kWgFaces - 1) / kWgFaces);
        if (!rc) rc = h->alloc(&L.wpart, (int64_t)nchunk * kNParam);
        if (rc) return rc;
    }
    rc = lic_adjoint_streams(h, st);
    if (rc) return rc;
    const int32_t saved_prec = h->precision, saved_active = L.active;
    h->precision = DD_FP64;
    L.active = 1;
    // the Q probes' applies in one launch each (grid.y = probe)
    hipError_t e = launch_apply_batch(h, R, L.Z, Q, st);
    L.active = saved_active;
    const int gres = (int)std::min<int64_t>((m + 255) / 256, 2048);
    if (e == hipSuccess) {
        k_lic_residual<<<dim3(gres, Q), 256, 0, st>>>(m, L.Z, Zs, den, Q, L.G, L.rpart, 2048);
        k_lic_loss<<<1, kLossT, 0, st>>>(Q, gres, 2048, L.rpart, den, loss);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_apply_adjoint(h, L.G, L.A, Q, st);
    h->precision = saved_prec;
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic applies: %s", hipGetErrorString(e));
    if (L.nf) {
        k_lic_dC<<<(unsigned)((L.nf * 9 + 255) / 256), 256, 0, st>>>(L.nf, m, Q, L.fI, L.fJ, L.A, R, L.dC);
        k_mlp_backprop<<<mlp_blocks(L.nf), 256, 0, st>>>(L.nf, params, L.dC, L.H1, L.H2, L.G1, L.G2);
        const int nchunk = (int)((L.nf + kWgFaces - 1) / kWgFaces);
        k_wgrad_mfma<<<dim3(nchunk, (kWgTiles + 3) / 4), 256, 0, st>>>(L.nf, L.dC, L.G2, L.G1, L.H2, L.H1, L.X,
                                                                        L.wpart);
        k_wgrad_sum<<<(kNParam + 255) / 256, 256, 0, st>>>(nchunk, L.wpart, grad, accumulate);
    } else if (!accumulate) {
        e = hipMemsetAsync(grad, 0, kNParam * sizeof(float), st);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic gradient: %s", hipGetErrorString(e));
    return DD_OK;
}

int lic_targets_run(dd_ctx *h, int Q, const double *R, double *Zs, double *den, hipStream_t st) {
    const int64_t m = h->n * 3;
    double *zdd = nullptr;
    int rc = h->alloc(&zdd, Q * m);
    if (rc) return rc;
    const int32_t saved_prec = h->precision;
    const int32_t saved_active = h->lic.active;
    h->precision = DD_FP64;
    h->lic.active = 0;
    hipError_t e = launch_global_apply(h, R, Zs, Q, st);
    if (e == hipSuccess) e = launch_apply_batch(h, R, zdd, Q, st);
    h->precision = saved_prec;
    h->lic.active = saved_active;
    if (e == hipSuccess) {
        k_lic_den<<<Q, 256, 0, st>>>(m, zdd, Zs, den);
        e = hipStreamSynchronize(st);
    }
    h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void *)zdd));
    (void)hipFree(zdd);
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic targets: %s", hipGetErrorString(e));
    return DD_OK;
}

hipError_t launch_adam(int np, float *P, const float *G, float *M, float *V, int t, float lr, float b1, float b2,
                       float eps, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    k_adam<<<(np + 255) / 256, 256, 0, st>>>(np, P, G, M, V, c1, c2, lr, b1, b2, eps);
    return hipGetLastError();
}

}  // namespace ddilu
