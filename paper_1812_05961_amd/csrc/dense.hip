// Dense FP64 steps of CP-ALS (Algorithm 1, Section III):
//   Gram  G = A^T A                       (the A^T A products)  -- FP64 MFMA
//   V     Hadamard of the other Grams
//   solve A = Y V^+   -- V^{-1} by symmetric Gauss-Jordan elimination (its
//         pivots are Cholesky's squared diagonal; the paper's code uses
//         potrf/potrs, Section V-A), or the Moore-Penrose inverse from a Jacobi
//         eigendecomposition when a pivot is <= R*eps*max(diag V)
//   norms lambda_r = ||A(:, r)||_2, unit columns
//   fit   1 - ||X - K|| / ||X||
#include "common.h"

namespace cpd {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GRAM_MAX_BLOCKS = 512;
constexpr double EPS64 = 2.220446049250313080847e-16;

struct GramSet {
    const double *g[CPD_MAX_MODES];
};

// ------------------------------------------------------------------ Gram
// Each wave accumulates the 16x16 blocks (bi <= bj) of A^T A over chunks of 4
// rows with v_mfma_f64_16x16x4f64: operand lane l holds A[row0 + l/16][16*b + l%16],
// which is element (l%16, l/16) of the 16x4 A^T slice and element (l/16, l%16)
// of the 4x16 A slice; result register v of lane l holds D[4*v + l/16][l%16].
template <int RB>
__global__ void __launch_bounds__(256)
k_gram(const float *__restrict__ A, int64_t rows, int R, int64_t ld, double *__restrict__ partial) {
    constexpr int P = RB * 16;
    __shared__ double red[P * P];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int krow = lane >> 4, kcol = lane & 15;
    v4d acc[RB][RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int64_t nchunks = ceil_div(rows, 4);
    for (int64_t ch = (int64_t)blockIdx.x * 4 + wave; ch < nchunks; ch += (int64_t)gridDim.x * 4) {
        const int64_t r = ch * 4 + krow;
        double f[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int col = b * 16 + kcol;
            f[b] = (r < rows && col < R) ? (double)A[r * ld + col] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = i; j < RB; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[i], f[j], acc[i][j], 0, 0, 0);
    }
    // deterministic reduction over the four waves
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = i; j < RB; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int rr = i * 16 + 4 * v + (lane >> 4), cc = j * 16 + (lane & 15);
                        if (w == 0) red[rr * P + cc] = acc[i][j][v];
                        else red[rr * P + cc] += acc[i][j][v];
                    }
        }
        __syncthreads();
    }
    double *out = partial + (int64_t)blockIdx.x * P * P;
    for (int t = threadIdx.x; t < P * P; t += 256) {
        const int rr = t / P, cc = t % P;
        out[t] = ((rr >> 4) <= (cc >> 4)) ? red[t] : 0.0;
    }
}

// sum over b < nb of p[b * stride] by one wave: lane l adds the terms
// b = l, l + 64, ... (independent loads), then a fixed butterfly combines the
// lanes, so the result is deterministic; every lane returns the total.
__device__ inline double wave_sum_strided(const double *__restrict__ p, int nb, int64_t stride) {
    const int lane = threadIdx.x & 63;
    double a = 0.0;
    for (int b = lane; b < nb; b += 64) a += p[(int64_t)b * stride];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    return a;
}

// Sum the per-block partials, one wave per entry; fill both triangles.
__global__ void __launch_bounds__(256) k_gram_reduce(const double *__restrict__ partial, int nblocks, int P, int R,
                                                     double *__restrict__ G) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= R * R) return;
    int r = t / R, c = t % R;
    const int rr = min(r, c), cc = max(r, c);
    // within a diagonal block both triangles were computed; outside, use the upper block
    const int src = ((rr >> 4) == (cc >> 4)) ? (r * P + c) : (rr * P + cc);
    const double v = wave_sum_strided(partial + src, nblocks, (int64_t)P * P);
    if ((threadIdx.x & 63) == 0) G[t] = v;
}

cpd_status gram(const float *A, int64_t rows, int R, int64_t ld, double *G, hipStream_t s) {
    if (!A || !G) CPD_FAIL(CPD_EINVAL, "null argument");
    if (R < 1 || R > CPD_MAX_RANK || ld < R || rows < 0) CPD_FAIL(CPD_EINVAL, "bad gram sizes");
    const int RB = (R + 15) / 16, P = RB * 16;
    int nb = (int)std::min<int64_t>(GRAM_MAX_BLOCKS, std::max<int64_t>(1, ceil_div(rows, 4 * 4 * 8)));
    DevBuf<double> part;
    CPD_TRY(part.alloc((size_t)nb * P * P, s));
    switch (RB) {
        case 1: hipLaunchKernelGGL(k_gram<1>, dim3(nb), dim3(256), 0, s, A, rows, R, ld, part.p); break;
        case 2: hipLaunchKernelGGL(k_gram<2>, dim3(nb), dim3(256), 0, s, A, rows, R, ld, part.p); break;
        case 3: hipLaunchKernelGGL(k_gram<3>, dim3(nb), dim3(256), 0, s, A, rows, R, ld, part.p); break;
        default: hipLaunchKernelGGL(k_gram<4>, dim3(nb), dim3(256), 0, s, A, rows, R, ld, part.p); break;
    }
    CPD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)ceil_div(R * R, 4)), dim3(256), 0, s,
                       (const double *)part.p, nb, P, R, G);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

// ------------------------------------------------------------------ W = V^+
// One block of NT threads: 256 when R^2 <= 256, else 1024.  The elimination
// runs R dependent steps of a few instructions per matrix entry, so above
// R = 16 sixteen waves (four per SIMD) hide each other's instruction and LDS
// latency (one wave per SIMD left every step latency-bound, about 2,900
// cycles at R = 35).  V (R x R, FP64) lives in LDS, built from the upper
// triangles of the Grams so that it is exactly symmetric; the fallback's
// eigenvectors in global scratch `wk` (R^2 doubles).  Writes W = V^{-1}
// (symmetric Gauss-Jordan) or V^+ (Jacobi eigendecomposition) to W, and the
// fallback flag.
template <int NT>
__global__ void __launch_bounds__(NT)
k_make_w(GramSet gs, int nmodes, int mode, int R, double *__restrict__ W, double *__restrict__ wk,
         int32_t *__restrict__ used_pinv) {
    __shared__ double V[CPD_MAX_RANK * CPD_MAX_RANK];
    __shared__ double sh[4];
    __shared__ int fail;
    const int tid = threadIdx.x;
    auto load_v = [&]() {
        for (int t = tid; t < R * R; t += NT) {
            const int r = t / R, c = t % R;
            const int u = min(r, c) * R + max(r, c);
            double v = 1.0;
            for (int m = 0; m < nmodes; ++m)
                if (m != mode) v *= gs.g[m][u];
            V[t] = v;
        }
        __syncthreads();
    };
    load_v();
    if (tid < 64) {  // wave 0: largest diagonal entry
        double mx = 0.0;
        for (int r = tid; r < R; r += 64) mx = fmax(mx, V[r * R + r]);
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if (tid == 0) {
            sh[0] = (double)R * EPS64 * mx;
            fail = 0;
        }
    }
    __syncthreads();
    const double thresh = sh[0];
    // W = V^{-1} by symmetric Gauss-Jordan elimination in place (the sweep
    // operator, Goodnight 1979; no pivoting, as for Cholesky on an SPD matrix).
    // Pivot j is the j-th diagonal of the Schur complement, the square of
    // Cholesky's L(j, j), so the same threshold decides between the inverse
    // and the fallback.  Sweeping every index leaves -V^{-1}; the update is
    // symmetric term by term, so W is exactly symmetric.
    // Two LDS copies: step j reads one and writes the other (one barrier per
    // step); each thread keeps the same entries for every step.  A step first
    // issues all of the thread's LDS reads (its entry and the two pivot-row
    // entries of each), then selects the result without branches: the reads
    // of a step overlap instead of each waiting out the LDS latency.  V stays
    // exactly symmetric, so the pivot column is read as the pivot row:
    // consecutive lanes then read consecutive words (a column read at R = 64
    // puts every lane of a wave in one LDS bank).
    __shared__ double Vs[2][CPD_MAX_RANK * CPD_MAX_RANK];
    constexpr int MAXE = CPD_MAX_RANK * CPD_MAX_RANK / NT;
    const int RR = R * R;
    const int ne = (RR + NT - 1) / NT;  // entry slots in use (block-uniform)
    int rr[MAXE], cc[MAXE];
#pragma unroll
    for (int i = 0; i < MAXE; ++i) {
        const int t = tid + NT * i;
        const bool in = t < RR;
        rr[i] = in ? t / R : 0;
        cc[i] = in ? t % R : 0;
        if (in) Vs[0][t] = V[t];
    }
    __syncthreads();
    bool ok = true;
    for (int j = 0; j < R; ++j) {
        const double *Vc = Vs[j & 1];
        double *Vn = Vs[(j + 1) & 1];
        const double d = Vc[j * R + j];
        if (!(d > thresh)) {
            ok = false;  // every thread reads the same d
            break;
        }
        double cur[MAXE], pr[MAXE], pc[MAXE];
#pragma unroll
        for (int i = 0; i < MAXE; ++i) {
            if (i < ne) {
                const int t = tid + NT * i;
                cur[i] = Vc[t < RR ? t : 0];
                pr[i] = Vc[j * R + rr[i]];
                pc[i] = Vc[j * R + cc[i]];
            }
        }
        const double inv = 1.0 / d;
#pragma unroll
        for (int i = 0; i < MAXE; ++i) {
            const int t = tid + NT * i;
            if (i < ne && t < RR) {
                const int r = rr[i], c = cc[i];
                double x = cur[i] - pr[i] * pc[i] * inv;
                x = (c == j) ? pr[i] * inv : x;
                x = (r == j) ? pc[i] * inv : x;
                x = (r == j && c == j) ? -inv : x;
                Vn[t] = x;
            }
        }
        __syncthreads();
    }
    if (ok) {
        const double *Vf = Vs[R & 1];
        for (int t = tid; t < R * R; t += NT) W[t] = -Vf[t];
        if (tid == 0 && used_pinv) *used_pinv = 0;
        return;
    }
    // Fallback: cyclic Jacobi on V (A <- J^T A J, Q <- Q J), Golub & Van Loan 8.4.
    __syncthreads();
    load_v();
    double *Q = wk;
    for (int t = tid; t < R * R; t += NT) Q[t] = (t / R == t % R) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) {
            double off = 0.0, tot = 0.0;
            for (int t = 0; t < R * R; ++t) {
                tot += V[t] * V[t];
                if (t / R != t % R) off += V[t] * V[t];
            }
            fail = (off <= EPS64 * EPS64 * tot) ? 2 : 1;
        }
        __syncthreads();
        if (fail == 2) break;
        for (int p = 0; p < R - 1; ++p) {
            for (int q = p + 1; q < R; ++q) {
                if (tid == 0) {
                    double apq = V[p * R + q];
                    double c = 1.0, s = 0.0;
                    if (apq != 0.0) {
                        double tau = (V[q * R + q] - V[p * R + p]) / (2.0 * apq);
                        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                    sh[1] = c;
                    sh[2] = s;
                }
                __syncthreads();
                const double c = sh[1], s = sh[2];
                if (s != 0.0) {
                    for (int k = tid; k < R; k += NT) {  // columns p, q
                        double akp = V[k * R + p], akq = V[k * R + q];
                        V[k * R + p] = c * akp - s * akq;
                        V[k * R + q] = s * akp + c * akq;
                        double qkp = Q[k * R + p], qkq = Q[k * R + q];
                        Q[k * R + p] = c * qkp - s * qkq;
                        Q[k * R + q] = s * qkp + c * qkq;
                    }
                    __syncthreads();
                    for (int k = tid; k < R; k += NT) {  // rows p, q
                        double apk = V[p * R + k], aqk = V[q * R + k];
                        V[p * R + k] = c * apk - s * aqk;
                        V[q * R + k] = s * apk + c * aqk;
                    }
                }
                __syncthreads();
            }
        }
    }
    if (tid == 0) {
        double wmax = -INFINITY;
        for (int r = 0; r < R; ++r) wmax = fmax(wmax, V[r * R + r]);
        sh[3] = (double)R * EPS64 * wmax;
    }
    __syncthreads();
    const double cut = sh[3];
    for (int t = tid; t < R * R; t += NT) {
        const int r = t / R, c = t % R;
        double x = 0.0;
        for (int k = 0; k < R; ++k) {
            double w = V[k * R + k];
            if (w > cut) x += Q[r * R + k] * Q[c * R + k] / w;
        }
        W[t] = x;
    }
    if (tid == 0 && used_pinv) *used_pinv = 1;
}

// A' = Y W (FP64) with v_mfma_f64_16x16x4f64: one wave per 16-row tile,
// NB = RP/16 column blocks, W zero-padded to RP x RP in LDS.  First operand
// lane l: Y[row0 + l%16][k0 + l/16]; second: W[k0 + l/16][16 nb + l%16];
// result register v of lane l: A'[row0 + 4v + l/16][16 nb + l%16].
// Pass 0 writes per-block column sums of squares, pass 1 the scaled rows
// (FP32 master and, when asked, the bfloat16 copy).
template <int RP>
__global__ void __launch_bounds__(256)
k_apply_w(const float *__restrict__ Y, int64_t rows, int R, int64_t ldy, const double *__restrict__ Wg,
          const double *__restrict__ lambda, float *__restrict__ A, int64_t lda,
          uint16_t *__restrict__ Ab, int64_t ldb, double *__restrict__ partial, int pass) {
    constexpr int NB = RP / 16;
    __shared__ double W[RP * RP];
    __shared__ double red[4][RP];
    for (int t = threadIdx.x; t < RP * RP; t += 256) {
        const int r = t / RP, c = t % RP;
        W[t] = (r < R && c < R) ? Wg[r * R + c] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    const int64_t arow = row0 + lr;  // row of this lane's first-operand element
    v4d acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < RP; k0 += 4) {
        const int k = k0 + lk;
        const double a = (arow < rows && k < R) ? (double)Y[arow * ldy + k] : 0.0;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, W[k * RP + nb * 16 + lr], acc[nb], 0, 0, 0);
    }
    if (pass == 0) {
        // column sums of squares: the 4 rows of each register, then the 4 lane
        // quarters holding the same column, then the 4 waves (fixed order)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            double q = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) q = fma(acc[nb][v], acc[nb][v], q);
            q += __shfl_xor(q, 16, 64);
            q += __shfl_xor(q, 32, 64);
            if (lk == 0) red[wave][nb * 16 + lr] = q;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < R; c += 256)
            partial[(int64_t)blockIdx.x * R + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
        return;
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int c = nb * 16 + lr;
        if (c >= R) continue;
        const double lam = lambda[c];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = row0 + 4 * v + lk;
            if (i >= rows) continue;
            const float x = lam > 0.0 ? (float)(acc[nb][v] / lam) : 0.0f;
            A[i * lda + c] = x;
            if (Ab) Ab[i * ldb + c] = f32_to_bf16(x);
        }
    }
}

__global__ void __launch_bounds__(256) k_lambda(const double *__restrict__ partial, int nblocks, int R,
                                                double *__restrict__ lambda) {
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);  // one wave per column
    if (c >= R) return;
    const double v = wave_sum_strided(partial + c, nblocks, R);
    if ((threadIdx.x & 63) == 0) lambda[c] = sqrt(v);
}

// ------------------------------------------------------------------ fit
// partial[b][r] = sum over this block's rows of A(i, r) * Y(i, r) (Y float,
// or double for the exact fit pass)
template <typename YT>
__global__ void __launch_bounds__(256)
k_fit_partial(const float *__restrict__ A, int64_t lda, const YT *__restrict__ Y, int64_t ldy,
              int64_t rows, int R, double *__restrict__ partial) {
    __shared__ double red[4][64];
    const int r = threadIdx.x & 63, grp = threadIdx.x >> 6;
    double s = 0.0;
    if (r < R)
        for (int64_t i = (int64_t)blockIdx.x * 4 + grp; i < rows; i += (int64_t)gridDim.x * 4)
            s += (double)A[i * lda + r] * (double)Y[i * ldy + r];
    red[grp][r] = s;
    __syncthreads();
    if (threadIdx.x < R)
        partial[(int64_t)blockIdx.x * R + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ void k_fit_final(const double *__restrict__ partial, int nblocks, int R,
                            const double *__restrict__ lambda, GramSet gs, int nmodes, double normX2,
                            double *__restrict__ fit) {
    __shared__ double inner_r[CPD_MAX_RANK], quad_r[CPD_MAX_RANK];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    // one wave per r: the column's partials, then sum_c lambda_r lambda_c prod_m G_m(r, c)
    for (int r = wave; r < R; r += nw) {
        const double in = wave_sum_strided(partial + r, nblocks, R);
        double q = 0.0;
        if (lane < R) {
            double h = 1.0;
            for (int m = 0; m < nmodes; ++m) h *= gs.g[m][r * R + lane];
            q = h * lambda[lane];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
        if (lane == 0) {
            inner_r[r] = lambda[r] * in;
            quad_r[r] = lambda[r] * q;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double inner = 0.0, normK2 = 0.0;
        for (int c = 0; c < R; ++c) {
            inner += inner_r[c];
            normK2 += quad_r[c];
        }
        double resid = normX2 - 2.0 * inner + normK2;
        resid = resid > 0.0 ? resid : 0.0;
        *fit = 1.0 - sqrt(resid) / sqrt(normX2);
    }
}

__global__ void __launch_bounds__(256)
k_sumsq_partial(const float *__restrict__ v, int64_t n, double *__restrict__ partial) {
    __shared__ double red[4];
    double s = 0.0;
    const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x, nt = (int64_t)gridDim.x * 256;
    if ((reinterpret_cast<uintptr_t>(v) & 15) == 0) {
        // 16-byte loads: four values per thread and step, the tail one by one
        const int64_t n4 = n >> 2;
        const float4 *v4 = reinterpret_cast<const float4 *>(v);
        for (int64_t i = tid; i < n4; i += nt) {
            const float4 q = v4[i];
            s += (double)q.x * q.x;
            s += (double)q.y * q.y;
            s += (double)q.z * q.z;
            s += (double)q.w * q.w;
        }
        for (int64_t i = (n4 << 2) + tid; i < n; i += nt) s += (double)v[i] * v[i];
    } else {
        for (int64_t i = tid; i < n; i += nt) s += (double)v[i] * v[i];
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// One wave: the sum of n partials in a fixed order.
__global__ void __launch_bounds__(64) k_sum_partials(const double *__restrict__ partial, int n,
                                                     double *__restrict__ out) {
    const double s = wave_sum_strided(partial, n, 1);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace

cpd_status gram_internal(const float *A, int64_t rows, int R, int64_t ld, double *G, hipStream_t s) {
    return gram(A, rows, R, ld, G, s);
}

cpd_status solve_normalize(const double *const *grams, int nmodes, int mode, const float *Y, int64_t rows,
                           int R, int64_t ldy, float *A, int64_t lda, uint16_t *Ab, int64_t ldb,
                           double *lambda, double *G_new, int32_t *used_pinv, hipStream_t s) {
    if (nmodes < 2 || nmodes > CPD_MAX_MODES || mode < 0 || mode >= nmodes)
        CPD_FAIL(CPD_EINVAL, "bad mode %d of %d", mode, nmodes);
    if (R < 1 || R > CPD_MAX_RANK || rows < 0 || ldy < R || lda < R || (Ab && ldb < R))
        CPD_FAIL(CPD_EINVAL, "bad solve sizes");
    if (!grams || !Y || !A || !lambda) CPD_FAIL(CPD_EINVAL, "null argument");
    GramSet gs{};
    for (int m = 0; m < nmodes; ++m) {
        if (m != mode && !grams[m]) CPD_FAIL(CPD_EINVAL, "null gram for mode %d", m);
        gs.g[m] = grams[m];
    }
    DevBuf<double> W, wk, part;
    CPD_TRY(W.alloc((size_t)R * R, s));
    CPD_TRY(wk.alloc((size_t)R * R, s));
    if (R * R <= 256)
        hipLaunchKernelGGL(k_make_w<256>, dim3(1), dim3(256), 0, s, gs, nmodes, mode, R, W.p, wk.p, used_pinv);
    else
        hipLaunchKernelGGL(k_make_w<1024>, dim3(1), dim3(1024), 0, s, gs, nmodes, mode, R, W.p, wk.p, used_pinv);
    CPD_LAUNCH_CHECK();
    const int nb = (int)std::max<int64_t>(1, ceil_div(rows, 64));  // 4 waves x 16 rows
    CPD_TRY(part.alloc((size_t)nb * R, s));
    const int RP = ((R + 15) / 16) * 16;
    for (int pass = 0; pass < 2; ++pass) {
#define CPD_APPLY(rp)                                                                                   \
    case rp:                                                                                            \
        hipLaunchKernelGGL(k_apply_w<rp>, dim3(nb), dim3(256), 0, s, Y, rows, R, (int64_t)ldy,          \
                           (const double *)W.p, (const double *)lambda, A, (int64_t)lda, Ab, (int64_t)ldb, \
                           part.p, pass);                                                               \
        break;
        switch (RP) {
            CPD_APPLY(16)
            CPD_APPLY(32)
            CPD_APPLY(48)
            CPD_APPLY(64)
        }
#undef CPD_APPLY
        CPD_LAUNCH_CHECK();
        if (pass == 0) {
            hipLaunchKernelGGL(k_lambda, dim3((unsigned)ceil_div(R, 4)), dim3(256), 0, s, (const double *)part.p, nb,
                               R, lambda);
            CPD_LAUNCH_CHECK();
        }
    }
    if (G_new) CPD_TRY(gram(A, rows, R, lda, G_new, s));
    return CPD_OK;
}

template <typename YT>
static cpd_status fit_t(double normX2, const double *lambda, const float *A, int64_t lda, const YT *Y, int64_t ldy,
                        int64_t rows, int R, const double *const *grams, int nmodes, double *out, hipStream_t s) {
    if (!lambda || !A || !Y || !grams || !out) CPD_FAIL(CPD_EINVAL, "null argument");
    if (R < 1 || R > CPD_MAX_RANK || nmodes < 2 || nmodes > CPD_MAX_MODES || lda < R || ldy < R)
        CPD_FAIL(CPD_EINVAL, "bad fit sizes");
    if (!(normX2 > 0.0)) CPD_FAIL(CPD_EINVAL, "||X||^2 must be positive");
    GramSet gs{};
    for (int m = 0; m < nmodes; ++m) {
        if (!grams[m]) CPD_FAIL(CPD_EINVAL, "null gram for mode %d", m);
        gs.g[m] = grams[m];
    }
    const int nb = (int)std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(rows, 64)));
    DevBuf<double> part;
    CPD_TRY(part.alloc((size_t)nb * R, s));
    hipLaunchKernelGGL(k_fit_partial<YT>, dim3(nb), dim3(256), 0, s, A, lda, Y, ldy, rows, R, part.p);
    CPD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fit_final, dim3(1), dim3(1024), 0, s, (const double *)part.p, nb, R, lambda, gs, nmodes,
                       normX2, out);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

cpd_status fit(double normX2, const double *lambda, const float *A, int64_t lda, const float *Y,
               int64_t ldy, int64_t rows, int R, const double *const *grams, int nmodes, double *out,
               hipStream_t s) {
    return fit_t<float>(normX2, lambda, A, lda, Y, ldy, rows, R, grams, nmodes, out, s);
}

// The fit from an FP64 MTTKRP of the last mode: <X, K> then carries FP64
// rounding only, so the residual keeps its accuracy as the fit nears 1.
cpd_status fit64(double normX2, const double *lambda, const float *A, int64_t lda, const double *Y,
                 int64_t ldy, int64_t rows, int R, const double *const *grams, int nmodes, double *out,
                 hipStream_t s) {
    return fit_t<double>(normX2, lambda, A, lda, Y, ldy, rows, R, grams, nmodes, out, s);
}

cpd_status sumsq(const float *v, int64_t n, double *out, hipStream_t s) {
    if (!v || !out || n < 0) CPD_FAIL(CPD_EINVAL, "bad sumsq arguments");
    const int nb = (int)std::min<int64_t>(2048, std::max<int64_t>(1, ceil_div(n, 1024)));
    DevBuf<double> part;
    CPD_TRY(part.alloc(nb, s));
    hipLaunchKernelGGL(k_sumsq_partial, dim3(nb), dim3(256), 0, s, v, n, part.p);
    CPD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, (const double *)part.p, nb, out);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

}  // namespace cpd

extern "C" {

cpd_status cpd_gram(const float *A, int64_t rows, int32_t rank, int32_t ld, double *G, void *stream) {
    cpd::clear_error();
    return cpd::gram_internal(A, rows, rank, ld, G, (hipStream_t)stream);
}

cpd_status cpd_solve_normalize(const double *const *grams, int32_t nmodes, int32_t mode, const float *Y,
                               int64_t rows, int32_t rank, int32_t ldy, float *A, int32_t lda,
                               uint16_t *A_bf16, int32_t ldb, double *lambda, double *G_new,
                               int32_t *used_pinv, void *stream) {
    cpd::clear_error();
    return cpd::solve_normalize(grams, nmodes, mode, Y, rows, rank, ldy, A, lda, A_bf16, ldb, lambda, G_new,
                                used_pinv, (hipStream_t)stream);
}

cpd_status cpd_fit(double normX2, const double *lambda, const float *A_last, int32_t lda, const float *Y_last,
                   int32_t ldy, int64_t rows, int32_t rank, const double *const *grams, int32_t nmodes,
                   double *fit, void *stream) {
    cpd::clear_error();
    return cpd::fit(normX2, lambda, A_last, lda, Y_last, ldy, rows, rank, grams, nmodes, fit, (hipStream_t)stream);
}

cpd_status cpd_sumsq(const float *vals, int64_t n, double *out, void *stream) {
    cpd::clear_error();
    return cpd::sumsq(vals, n, out, (hipStream_t)stream);
}

}  // extern "C"
