// Message-passing network for the learned initial displacement guess:
// forward, backward (hand-written adjoints) and Adam, float32, on the vertex
// graph of a P1 mesh.  The paper starts each transient solve from the previous
// step's displacement (Sec. 5.3); here the starting guess comes from the load.
//
//   h0   = relu(X W_in + b_in)                               X: [N, 10]
//   for l < 4:  m = mean_{u in N(v)} h_u;  g = mean_v h_v
//               d_k = sum_{u in N(v)} w^k_vu h_u   (k = x, y, z)
//               h = h + relu(h W_s + m W_n + g W_g + d_x W_dx + d_y W_dy + d_z W_dz + b)
//   y    = (h W_out + b_out) * (1 - mask)                    [N, 3]
// with the direction weights w^k_vu = (x_u - x_v)_k / (deg_v l_v), l_v the
// mean length of the edges at v (a first-difference stencil).
//
// Layouts: activations [N][64] row-major, the directional sums [N][3][64];
// parameters one float array in the order W_in[10][64], b_in[64], per layer
// {W_s, W_n, W_g, W_dx, W_dy, W_dz}[64][64], b[64], W_out[64][3], b_out[3]
// (weights [in][out]), so the three directional weights of a layer form one
// [192][64] matrix against the [N][192] sums.
//
// Vertex kernels run one wave per vertex with the 64 channels on the lanes
// (the neighbour gather is then a coalesced 256-byte row read; a vertex's
// channel values reach every lane by readlane); weight gradients X^T Y are
// blocked reductions over vertices with per-block partial tiles summed in a
// fixed order (deterministic, no atomics).  The graph is symmetric, so the
// adjoints of the neighbour mean and of the directional sums are gathers
// too: d h_u = sum_{v in N(u)} (d m_v / deg_v + sum_k w^k_vu d d_k[v]).
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>

#include "te_amg.h"
#include "te_internal.h"

namespace te {

constexpr int MH = 64, ML = 4, MF = 10, MO = 3, MD = 3 * MH;
constexpr int64_t OFF_WIN = 0, OFF_BIN = MF * MH;
constexpr int64_t LAYER0 = OFF_BIN + MH;
constexpr int64_t LAYER_SZ = 6 * MH * MH + MH;
constexpr int64_t OFF_WOUT = LAYER0 + ML * LAYER_SZ;
constexpr int64_t OFF_BOUT = OFF_WOUT + MH * MO;
constexpr int64_t NPARAM = OFF_BOUT + MO;
constexpr float S_T = 500.f, S_F = 2.0e9f, S_X = 0.5f;
constexpr double S_U = 1.0e-3;
constexpr int MB = 256, MW = MB / 64;
constexpr int VB = 4;   // vertices per wave step of the dense layer transforms
constexpr int RED_BLOCKS = 512;

__host__ __device__ constexpr int64_t off_ws(int l) { return LAYER0 + l * LAYER_SZ; }
__host__ __device__ constexpr int64_t off_wn(int l) { return LAYER0 + l * LAYER_SZ + MH * MH; }
__host__ __device__ constexpr int64_t off_wg(int l) { return LAYER0 + l * LAYER_SZ + 2 * MH * MH; }
__host__ __device__ constexpr int64_t off_wd(int l) { return LAYER0 + l * LAYER_SZ + 3 * MH * MH; }
__host__ __device__ constexpr int64_t off_b(int l) { return LAYER0 + l * LAYER_SZ + 6 * MH * MH; }

__device__ __forceinline__ float lane_val(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

static inline unsigned vgrid(int64_t n) {
    int64_t g = (n + MW - 1) / MW;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// features: X[v] = [dT/S_T, f/S_F, mask, xc/S_X]
__global__ void k_features(int64_t n, const double *__restrict__ xc, const double *__restrict__ T, double T_ref,
                           const double *__restrict__ f, const uint8_t *__restrict__ mask, float *__restrict__ X) {
    for (int64_t v = blockIdx.x * (int64_t)MB + threadIdx.x; v < n; v += (int64_t)gridDim.x * MB) {
        float *o = X + v * MF;
        o[0] = float((T[v] - T_ref) / S_T);
        for (int c = 0; c < 3; ++c) {
            o[1 + c] = f ? float(f[v * 3 + c] / S_F) : 0.f;
            o[4 + c] = mask[v * 3 + c] ? 1.f : 0.f;
            o[7 + c] = float(xc[v * 3 + c] / S_X);
        }
    }
}

// h0 = relu(X W_in + b_in): one wave per vertex, lane = channel
__global__ void __launch_bounds__(MB) k_in(int64_t n, const float *__restrict__ P, const float *__restrict__ X,
                                           float *__restrict__ h0) {
    const int c = threadIdx.x & 63;
    for (int64_t v = blockIdx.x * (int64_t)MW + threadIdx.x / 64; v < n; v += (int64_t)gridDim.x * MW) {
        float a = P[OFF_BIN + c];
        for (int k = 0; k < MF; ++k) a += X[v * MF + k] * P[OFF_WIN + k * MH + c];
        h0[v * MH + c] = a > 0.f ? a : 0.f;
    }
}

// column sums of an [n][64] array: partials[block][64]
__global__ void __launch_bounds__(MB) k_colsum(int64_t n, const float *__restrict__ H, double *__restrict__ part) {
    __shared__ double lds[MB];
    const int c = threadIdx.x & 63, w = threadIdx.x / 64;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double t = 0.0;
    for (int64_t v = lo + w; v < hi; v += MW) t += H[v * MH + c];
    lds[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int k = 0; k < MW; ++k) s += lds[k * 64 + threadIdx.x];
        part[blockIdx.x * 64 + threadIdx.x] = s;
    }
}

// g = colsum/n (from partials), gw = g W_g + b (forward) ; one block of 64
__global__ void k_global(int nparts, const double *__restrict__ part, int64_t n, const float *__restrict__ P, int l,
                         float *__restrict__ g, float *__restrict__ gw) {
    __shared__ float gs[64];
    const int c = threadIdx.x;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[b * 64 + c];
    gs[c] = float(s / double(n));
    g[c] = gs[c];
    __syncthreads();
    float a = P[off_b(l) + c];
    for (int k = 0; k < MH; ++k) a += gs[k] * P[off_wg(l) + k * MH + c];
    gw[c] = a;
}

// one message-passing layer: m = mean of neighbours, d = directional sums,
// a = h W_s + m W_n + d W_d + gw, h' = h + relu(a); stores m, d and a for the
// backward pass.  W_s, W_n, W_dx and W_dy sit in LDS (64 KB), W_dz is read
// through the cache; a wave takes VB vertices at a time, each weight value
// serving all of them.
__global__ void __launch_bounds__(MB) k_mp_fwd(int64_t n, const int64_t *__restrict__ gp, const int32_t *__restrict__ gi,
                                               const float *__restrict__ xf, const float *__restrict__ invdl,
                                               const float *__restrict__ P, int l, const float *__restrict__ gw,
                                               const float *__restrict__ h, float *__restrict__ m,
                                               float *__restrict__ d, float *__restrict__ a, float *__restrict__ hn) {
    extern __shared__ float W[];   // [4][64][64]: W_s, W_n, W_dx, W_dy
    for (int t = threadIdx.x; t < MH * MH; t += MB) {
        W[t] = P[off_ws(l) + t];
        W[MH * MH + t] = P[off_wn(l) + t];
    }
    for (int t = threadIdx.x; t < 2 * MH * MH; t += MB) W[2 * MH * MH + t] = P[off_wd(l) + t];
    __syncthreads();
    const float *__restrict__ Wz = P + off_wd(l) + 2 * MH * MH;
    const int c = threadIdx.x & 63;
    const float gwc = gw[c];
    const int64_t step = (int64_t)gridDim.x * MW * VB;
    for (int64_t v0 = (blockIdx.x * (int64_t)MW + threadIdx.x / 64) * VB; v0 < n; v0 += step) {
        float hv[VB], mv[VB], d0[VB], d1[VB], d2[VB], acc[VB];
#pragma unroll
        for (int i = 0; i < VB; ++i) {
            const int64_t v = v0 + i;
            hv[i] = mv[i] = d0[i] = d1[i] = d2[i] = 0.f;
            acc[i] = gwc;
            if (v >= n) continue;
            const int64_t lo = gp[v], hi = gp[v + 1];
            const float xv0 = xf[v * 3], xv1 = xf[v * 3 + 1], xv2 = xf[v * 3 + 2], iv = invdl[v];
            float s = 0.f;
            for (int64_t e = lo; e < hi; ++e) {
                const int64_t u = gi[e];
                const float hu = h[u * MH + c];
                s += hu;
                d0[i] += (xf[u * 3] - xv0) * iv * hu;
                d1[i] += (xf[u * 3 + 1] - xv1) * iv * hu;
                d2[i] += (xf[u * 3 + 2] - xv2) * iv * hu;
            }
            mv[i] = hi > lo ? s / float(hi - lo) : 0.f;
            hv[i] = h[v * MH + c];
        }
#pragma unroll 4
        for (int k = 0; k < MH; ++k) {
            const float ws = W[k * MH + c], wn = W[MH * MH + k * MH + c], wx = W[2 * MH * MH + k * MH + c],
                        wy = W[3 * MH * MH + k * MH + c], wz = Wz[k * MH + c];
#pragma unroll
            for (int i = 0; i < VB; ++i) {
                acc[i] += lane_val(hv[i], k) * ws;
                acc[i] += lane_val(mv[i], k) * wn;
                acc[i] += lane_val(d0[i], k) * wx;
                acc[i] += lane_val(d1[i], k) * wy;
                acc[i] += lane_val(d2[i], k) * wz;
            }
        }
#pragma unroll
        for (int i = 0; i < VB; ++i) {
            const int64_t v = v0 + i;
            if (v >= n) break;
            m[v * MH + c] = mv[i];
            d[v * MD + c] = d0[i];
            d[v * MD + MH + c] = d1[i];
            d[v * MD + 2 * MH + c] = d2[i];
            a[v * MH + c] = acc[i];
            hn[v * MH + c] = hv[i] + (acc[i] > 0.f ? acc[i] : 0.f);
        }
    }
}

// y = (h W_out + b_out) * keep ; if target: loss and gy = 2 (y - t)/(3n) * keep,
// gh = gy W_out^T ; per-block partial loss
__global__ void __launch_bounds__(MB) k_out(int64_t n, const float *__restrict__ P, const float *__restrict__ h,
                                            const uint8_t *__restrict__ mask, float *__restrict__ y,
                                            const float *__restrict__ target, float *__restrict__ gy,
                                            float *__restrict__ gh, double *__restrict__ lpart) {
    __shared__ double lds[MW];
    const int c = threadIdx.x & 63, w = threadIdx.x / 64;
    double lsum = 0.0;
    const float inv = 2.f / float(3 * n);
    for (int64_t v = blockIdx.x * (int64_t)MW + w; v < n; v += (int64_t)gridDim.x * MW) {
        const float hv = h[v * MH + c];
        float yv[MO];
        for (int j = 0; j < MO; ++j) {
            float t = hv * P[OFF_WOUT + c * MO + j];
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
            const float keep = mask[v * 3 + j] ? 0.f : 1.f;
            yv[j] = (t + P[OFF_BOUT + j]) * keep;
        }
        if (c < MO) y[v * MO + c] = c == 0 ? yv[0] : (c == 1 ? yv[1] : yv[2]);
        if (target) {
            float g[MO];
            for (int j = 0; j < MO; ++j) {
                const float keep = mask[v * 3 + j] ? 0.f : 1.f;
                const float d = yv[j] - target[v * MO + j];
                if (c == 0) lsum += double(d) * double(d);
                g[j] = inv * d * keep;
            }
            if (c < MO) gy[v * MO + c] = c == 0 ? g[0] : (c == 1 ? g[1] : g[2]);
            float ghc = 0.f;
            for (int j = 0; j < MO; ++j) ghc += g[j] * P[OFF_WOUT + c * MO + j];
            gh[v * MH + c] = ghc;
        }
    }
    if (target) {
        if (c == 0) lds[w] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int k = 0; k < MW; ++k) t += lds[k];
            lpart[blockIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// ga = gh * (a > 0); gmd = (ga W_n^T) / deg; gd_k = ga W_dk^T.  The four
// matrices sit transposed in LDS (64 KB), so lane c reads W[c][k] of row k
// of the copy: consecutive lanes, consecutive banks.  A wave takes VB
// vertices at a time, each LDS value serving all of them.

__global__ void __launch_bounds__(MB) k_mp_bwd1(int64_t n, const int64_t *__restrict__ gp, const float *__restrict__ P,
                                                int l, const float *__restrict__ gh, const float *__restrict__ a,
                                                float *__restrict__ ga, float *__restrict__ gmd,
                                                float *__restrict__ gd) {
    extern __shared__ float W[];   // [4][64][64] transposed: W_n, W_dx, W_dy, W_dz
    for (int t = threadIdx.x; t < MH * MH; t += MB) {
        const int r = t / MH, q = t % MH;   // W[r][q] -> copy[q][r]
        W[q * MH + r] = P[off_wn(l) + t];
        W[MH * MH + q * MH + r] = P[off_wd(l) + t];
        W[2 * MH * MH + q * MH + r] = P[off_wd(l) + MH * MH + t];
        W[3 * MH * MH + q * MH + r] = P[off_wd(l) + 2 * MH * MH + t];
    }
    __syncthreads();
    const int c = threadIdx.x & 63;
    const int64_t step = (int64_t)gridDim.x * MW * VB;
    for (int64_t v0 = (blockIdx.x * (int64_t)MW + threadIdx.x / 64) * VB; v0 < n; v0 += step) {
        float g[VB], t[VB][4];
#pragma unroll
        for (int i = 0; i < VB; ++i) {
            const int64_t v = v0 + i;
            g[i] = v < n && a[v * MH + c] > 0.f ? gh[v * MH + c] : 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) t[i][j] = 0.f;
        }
#pragma unroll 4
        for (int k = 0; k < MH; ++k) {
            // W^T[k][c] of each matrix: W[c][k] (row c of the weight, column k)
            const float w0 = W[k * MH + c], w1 = W[MH * MH + k * MH + c], w2 = W[2 * MH * MH + k * MH + c],
                        w3 = W[3 * MH * MH + k * MH + c];
#pragma unroll
            for (int i = 0; i < VB; ++i) {
                const float gk = lane_val(g[i], k);
                t[i][0] += gk * w0;
                t[i][1] += gk * w1;
                t[i][2] += gk * w2;
                t[i][3] += gk * w3;
            }
        }
#pragma unroll
        for (int i = 0; i < VB; ++i) {
            const int64_t v = v0 + i;
            if (v >= n) break;
            ga[v * MH + c] = g[i];
            const int64_t deg = gp[v + 1] - gp[v];
            gmd[v * MH + c] = deg > 0 ? t[i][0] / float(deg) : 0.f;
            gd[v * MD + c] = t[i][1];
            gd[v * MD + MH + c] = t[i][2];
            gd[v * MD + 2 * MH + c] = t[i][3];
        }
    }
}

// gh_prev = gh + ga W_s^T + gg / n + sum_{u in N(v)} (gmd_u + sum_k w^k_uv gd_k[u]),
// w^k_uv = (x_v - x_u)_k / (deg_u l_u)
__global__ void __launch_bounds__(MB) k_mp_bwd2(int64_t n, const int64_t *__restrict__ gp, const int32_t *__restrict__ gi,
                                                const float *__restrict__ xf, const float *__restrict__ invdl,
                                                const float *__restrict__ P, int l, const float *__restrict__ ga,
                                                const float *__restrict__ gmd, const float *__restrict__ gd,
                                                const float *__restrict__ gg, float *__restrict__ gh) {
    __shared__ float Ws[MH * MH];   // W_s transposed (conflict-free reads, as k_mp_bwd1)
    for (int t = threadIdx.x; t < MH * MH; t += MB) Ws[(t % MH) * MH + t / MH] = P[off_ws(l) + t];
    __syncthreads();
    const int c = threadIdx.x & 63;
    const float ggc = gg[c] / float(n);
    for (int64_t v = blockIdx.x * (int64_t)MW + threadIdx.x / 64; v < n; v += (int64_t)gridDim.x * MW) {
        const float g = ga[v * MH + c];
        float t = gh[v * MH + c] + ggc;
#pragma unroll 8
        for (int k = 0; k < MH; ++k) t += lane_val(g, k) * Ws[k * MH + c];
        const float xv0 = xf[v * 3], xv1 = xf[v * 3 + 1], xv2 = xf[v * 3 + 2];
        for (int64_t e = gp[v]; e < gp[v + 1]; ++e) {
            const int64_t u = gi[e];
            const float iu = invdl[u];
            t += gmd[u * MH + c];
            t += (xv0 - xf[u * 3]) * iu * gd[u * MD + c];
            t += (xv1 - xf[u * 3 + 1]) * iu * gd[u * MD + MH + c];
            t += (xv2 - xf[u * 3 + 2]) * iu * gd[u * MD + 2 * MH + c];
        }
        gh[v * MH + c] = t;
    }
}

// ga_in = gh * (h0 > 0)
__global__ void k_relu_mask(int64_t n, const float *__restrict__ h0, const float *__restrict__ gh,
                            float *__restrict__ ga) {
    for (int64_t t = blockIdx.x * (int64_t)MB + threadIdx.x; t < n * MH; t += (int64_t)gridDim.x * MB)
        ga[t] = h0[t] > 0.f ? gh[t] : 0.f;
}

// partial X^T Y over a chunk of vertices: X [n][KX], Y [n][KY]; block partial
// tile [KX][KY] (thread t owns entries t, t+256, ...)
template <int KX, int KY>
__global__ void __launch_bounds__(MB) k_xty(int64_t n, const float *__restrict__ X, const float *__restrict__ Y,
                                            float *__restrict__ part) {
    constexpr int ROWS = 32;
    __shared__ float xs[ROWS * KX], ys[ROWS * KY];
    constexpr int PER = (KX * KY + MB - 1) / MB;
    float acc[PER];
    for (int q = 0; q < PER; ++q) acc[q] = 0.f;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (int64_t r0 = lo; r0 < hi; r0 += ROWS) {
        const int rows = (int)min<int64_t>(ROWS, hi - r0);
        for (int t = threadIdx.x; t < ROWS * KX; t += MB) xs[t] = (t / KX) < rows ? X[(r0 + t / KX) * KX + t % KX] : 0.f;
        for (int t = threadIdx.x; t < ROWS * KY; t += MB) ys[t] = (t / KY) < rows ? Y[(r0 + t / KY) * KY + t % KY] : 0.f;
        __syncthreads();
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + q * MB;
            if (e < KX * KY) {
                const int i = e / KY, j = e % KY;
                float s = 0.f;
                for (int r = 0; r < rows; ++r) s += xs[r * KX + i] * ys[r * KY + j];
                acc[q] += s;
            }
        }
        __syncthreads();
    }
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * MB;
        if (e < KX * KY) part[blockIdx.x * (int64_t)(KX * KY) + e] = acc[q];
    }
}

// out[e] (+)= sum_b part[b][e], fixed order in double
__global__ void k_sum_parts(int nparts, int nel, const float *__restrict__ part, float *__restrict__ out) {
    for (int e = blockIdx.x * MB + threadIdx.x; e < nel; e += gridDim.x * MB) {
        double s = 0.0;
        for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * nel + e];
        out[e] = float(s);
    }
}

// layer scalars: gb = colsum(ga); gW_g = g^T gb (outer product); gg = gb W_g^T
__global__ void k_layer_small(int nparts, const double *__restrict__ part, const float *__restrict__ g,
                              const float *__restrict__ P, int l, float *__restrict__ grad, float *__restrict__ gg) {
    __shared__ float gb[64];
    const int c = threadIdx.x;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[b * 64 + c];
    gb[c] = float(s);
    grad[off_b(l) + c] = gb[c];
    __syncthreads();
    for (int k = 0; k < MH; ++k) grad[off_wg(l) + k * MH + c] = g[k] * gb[c];
    float t = 0.f;
    for (int k = 0; k < MH; ++k) t += gb[k] * P[off_wg(l) + c * MH + k];
    gg[c] = t;
}

// b grads from partial colsums of widths <= 64
__global__ void k_colsum_out(int nparts, const double *__restrict__ part, int width, float *__restrict__ out) {
    const int c = threadIdx.x;
    if (c >= width) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[b * 64 + c];
    out[c] = float(s);
}

// column sums of an [n][3] array into partials[block][64] (first 3 used)
__global__ void __launch_bounds__(MB) k_colsum3(int64_t n, const float *__restrict__ Y, double *__restrict__ part) {
    __shared__ double lds[MB * 3];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double t[3] = {0, 0, 0};
    for (int64_t v = lo + threadIdx.x; v < hi; v += MB)
        for (int j = 0; j < 3; ++j) t[j] += Y[v * 3 + j];
    for (int j = 0; j < 3; ++j) lds[threadIdx.x * 3 + j] = t[j];
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int k = 0; k < MB; ++k) s += lds[k * 3 + threadIdx.x];
        part[blockIdx.x * 64 + threadIdx.x] = s;
    }
}

// gh = (gy * keep) W_out^T, gy_masked stored
__global__ void __launch_bounds__(MB) k_gy_to_gh(int64_t n, const float *__restrict__ P, const uint8_t *__restrict__ mask,
                                                 const float *__restrict__ gy_in, float *__restrict__ gy,
                                                 float *__restrict__ gh) {
    const int c = threadIdx.x & 63;
    for (int64_t v = blockIdx.x * (int64_t)MW + threadIdx.x / 64; v < n; v += (int64_t)gridDim.x * MW) {
        float g[MO];
        for (int j = 0; j < MO; ++j) g[j] = mask[v * 3 + j] ? 0.f : gy_in[v * MO + j];
        if (c < MO) gy[v * MO + c] = c == 0 ? g[0] : (c == 1 ? g[1] : g[2]);
        float t = 0.f;
        for (int j = 0; j < MO; ++j) t += g[j] * P[OFF_WOUT + c * MO + j];
        gh[v * MH + c] = t;
    }
}

// u = S_U y * keep, u_t = S_U t  (float64, natural order)
__global__ void k_energy_prep(int64_t n, const float *__restrict__ y, const float *__restrict__ t,
                              const uint8_t *__restrict__ mask, double *__restrict__ u, double *__restrict__ ut) {
    for (int64_t i = blockIdx.x * (int64_t)MB + threadIdx.x; i < n * 3; i += (int64_t)gridDim.x * MB) {
        u[i] = mask[i] ? 0.0 : S_U * double(y[i]);
        ut[i] = S_U * double(t[i]);
    }
}
// gy = keep * (ca * A u_t + cb * A u)  (float)
__global__ void k_energy_gy(int64_t n, const double *__restrict__ Aut, const double *__restrict__ Au,
                            const uint8_t *__restrict__ mask, double ca, double cb, float *__restrict__ gy) {
    for (int64_t i = blockIdx.x * (int64_t)MB + threadIdx.x; i < n * 3; i += (int64_t)gridDim.x * MB)
        gy[i] = mask[i] ? 0.f : float(ca * Aut[i] + cb * Au[i]);
}

// Adam (Kingma & Ba 2015) with bias correction
__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)MB + threadIdx.x; i < n; i += (int64_t)gridDim.x * MB) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_guess(int64_t n, const float *__restrict__ y, double *__restrict__ u0) {
    for (int64_t t = blockIdx.x * (int64_t)MB + threadIdx.x; t < n * 3; t += (int64_t)gridDim.x * MB)
        u0[t] = S_U * double(y[t]);
}

// 1 / (deg_v l_v), l_v the mean length of the edges at v (0 without edges)
__global__ void k_invdl(int64_t n, const int64_t *__restrict__ gp, const int32_t *__restrict__ gi,
                        const double *__restrict__ xc, float *__restrict__ invdl, float *__restrict__ xf) {
    for (int64_t v = blockIdx.x * (int64_t)MB + threadIdx.x; v < n; v += (int64_t)gridDim.x * MB) {
        double len = 0.0;
        for (int64_t e = gp[v]; e < gp[v + 1]; ++e) {
            const int64_t u = gi[e];
            const double a = xc[u * 3] - xc[v * 3], b = xc[u * 3 + 1] - xc[v * 3 + 1], c = xc[u * 3 + 2] - xc[v * 3 + 2];
            len += sqrt(a * a + b * b + c * c);
        }
        const int64_t deg = gp[v + 1] - gp[v];
        invdl[v] = deg > 0 && len > 0.0 ? float(1.0 / len) : 0.f;   // 1 / (deg * (len / deg))
        for (int k = 0; k < 3; ++k) xf[v * 3 + k] = float(xc[v * 3 + k]);
    }
}

// vertex graph = stiffness pattern without the diagonal
__global__ void k_graph_count(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              int32_t *__restrict__ cnt) {
    for (int64_t v = blockIdx.x * (int64_t)MB + threadIdx.x; v < n; v += (int64_t)gridDim.x * MB) {
        int c = 0;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) c += ci[e] != v;
        cnt[v] = c;
    }
}
__global__ void k_graph_fill(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const int64_t *__restrict__ gp, int32_t *__restrict__ gi) {
    for (int64_t v = blockIdx.x * (int64_t)MB + threadIdx.x; v < n; v += (int64_t)gridDim.x * MB) {
        int64_t o = gp[v];
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
            if (ci[e] != v) gi[o++] = ci[e];
    }
}

}  // namespace te

// ---------------------------------------------------------------------------
// handle and C ABI
// ---------------------------------------------------------------------------
struct mpnn_handle {
    int64_t n = 0;
    te::DBuf<int64_t> gp;
    te::DBuf<int32_t> gi;
    te::DBuf<double> xc;  // centred coordinates
    te::DBuf<float> xf, invdl;  // float centred coordinates, 1 / (deg l) per vertex
    te::DBuf<float> h[te::ML + 1], m[te::ML], d[te::ML], a[te::ML], g[te::ML], gw;
    te::DBuf<float> y, gy, gh, ga, gmd, gd, gg, part;
    te::DBuf<double> dpart;
    te::DBuf<float> X;     // last forward input (borrowed copy)
    te::DBuf<uint8_t> mask;
    bool have_forward = false;
};

using namespace te;

extern "C" int64_t mpnn_param_count(void) { return NPARAM; }

extern "C" int mpnn_create(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *coords,
                           mpnn_handle **out, hipStream_t s) {
    return guarded([&] {
        TE_REQUIRE(n > 0 && row_ptr && col_idx && coords && out, TE_EINVAL, "bad argument");
        auto H = std::make_unique<mpnn_handle>();
        H->n = n;
        DBuf<int32_t> cnt(n);
        const unsigned g = (unsigned)std::min<int64_t>((n + MB - 1) / MB, 65536);
        hipLaunchKernelGGL(k_graph_count, dim3(g), dim3(MB), 0, s, n, row_ptr, col_idx, cnt.p);
        TE_CHECK_HIP(hipGetLastError());
        std::vector<int32_t> hc;
        download(hc, cnt.p, n, s);
        std::vector<int64_t> gp(n + 1, 0);
        for (int64_t v = 0; v < n; ++v) gp[v + 1] = gp[v] + hc[v];
        upload(H->gp, gp, s);
        H->gi.alloc(std::max<int64_t>(gp[n], 1));
        hipLaunchKernelGGL(k_graph_fill, dim3(g), dim3(MB), 0, s, n, row_ptr, col_idx, H->gp.p, H->gi.p);
        TE_CHECK_HIP(hipGetLastError());
        std::vector<double> X;
        download(X, coords, n * 3, s);
        double c[3] = {0, 0, 0};
        for (int64_t v = 0; v < n; ++v)
            for (int k = 0; k < 3; ++k) c[k] += X[v * 3 + k];
        for (int k = 0; k < 3; ++k) c[k] /= double(n);
        for (int64_t v = 0; v < n; ++v)
            for (int k = 0; k < 3; ++k) X[v * 3 + k] -= c[k];
        upload(H->xc, X, s);
        H->xf.alloc(n * 3);
        H->invdl.alloc(n);
        hipLaunchKernelGGL(k_invdl, dim3(g), dim3(MB), 0, s, n, H->gp.p, H->gi.p, H->xc.p, H->invdl.p, H->xf.p);
        TE_CHECK_HIP(hipGetLastError());
        for (int l = 0; l <= ML; ++l) H->h[l].alloc(n * MH);
        for (int l = 0; l < ML; ++l) {
            H->m[l].alloc(n * MH);
            H->d[l].alloc(n * MD);
            H->a[l].alloc(n * MH);
            H->g[l].alloc(MH);
        }
        H->gw.alloc(MH);
        H->y.alloc(n * MO);
        H->gy.alloc(n * MO);
        H->gh.alloc(n * MH);
        H->ga.alloc(n * MH);
        H->gmd.alloc(n * MH);
        H->gd.alloc(n * MD);
        H->gg.alloc(MH);
        H->part.alloc((size_t)RED_BLOCKS * MD * MH);
        H->dpart.alloc((size_t)RED_BLOCKS * 64);
        H->X.alloc(n * MF);
        H->mask.alloc(n * 3);
        TE_CHECK_HIP(hipStreamSynchronize(s));
        *out = H.release();
        return TE_OK;
    });
}

extern "C" int mpnn_destroy(mpnn_handle *h) {
    delete h;
    return TE_OK;
}

extern "C" int mpnn_features(mpnn_handle *H, const double *T, double T_ref, const double *f, const uint8_t *mask,
                             float *X, hipStream_t s) {
    return guarded([&] {
        TE_REQUIRE(H && T && mask && X, TE_EINVAL, "bad argument");
        const unsigned g = (unsigned)std::min<int64_t>((H->n + MB - 1) / MB, 65536);
        hipLaunchKernelGGL(k_features, dim3(g), dim3(MB), 0, s, H->n, H->xc.p, T, T_ref, f, mask, X);
        TE_CHECK_HIP(hipGetLastError());
        return TE_OK;
    });
}

static int nparts_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, (n + 255) / 256)); }

extern "C" int mpnn_forward(mpnn_handle *H, const float *P, const float *X, const uint8_t *mask, float *y,
                            hipStream_t s) {
    return guarded([&] {
        TE_REQUIRE(H && P && X && mask, TE_EINVAL, "bad argument");
        const int64_t n = H->n;
        TE_CHECK_HIP(hipMemcpyAsync(H->X.p, X, n * MF * sizeof(float), hipMemcpyDeviceToDevice, s));
        TE_CHECK_HIP(hipMemcpyAsync(H->mask.p, mask, n * 3, hipMemcpyDeviceToDevice, s));
        const int np = nparts_for(n);
        hipLaunchKernelGGL(k_in, dim3(vgrid(n)), dim3(MB), 0, s, n, P, X, H->h[0].p);
        for (int l = 0; l < ML; ++l) {
            hipLaunchKernelGGL(k_colsum, dim3(np), dim3(MB), 0, s, n, H->h[l].p, H->dpart.p);
            hipLaunchKernelGGL(k_global, dim3(1), dim3(64), 0, s, np, H->dpart.p, n, P, l, H->g[l].p, H->gw.p);
            hipLaunchKernelGGL(k_mp_fwd, dim3(vgrid((n + VB - 1) / VB)), dim3(MB), 4 * MH * MH * sizeof(float), s, n,
                               H->gp.p,
                               H->gi.p, H->xf.p, H->invdl.p, P, l, H->gw.p, H->h[l].p, H->m[l].p, H->d[l].p,
                               H->a[l].p, H->h[l + 1].p);
        }
        hipLaunchKernelGGL(k_out, dim3(vgrid(n)), dim3(MB), 0, s, n, P, H->h[ML].p, mask, y ? y : H->y.p,
                           (const float *)nullptr, (float *)nullptr, (float *)nullptr, (double *)nullptr);
        TE_CHECK_HIP(hipGetLastError());
        if (y && y != H->y.p) TE_CHECK_HIP(hipMemcpyAsync(H->y.p, y, n * MO * sizeof(float), hipMemcpyDeviceToDevice, s));
        H->have_forward = true;
        return TE_OK;
    });
}

static void backward_tail(mpnn_handle *H, const float *P, float *grad, hipStream_t s) {
    const int64_t n = H->n;
    const int np = nparts_for(n);
    const unsigned vg = vgrid(n);
    // output layer (gy and gh are in the handle)
    hipLaunchKernelGGL((k_xty<MH, MO>), dim3(np), dim3(MB), 0, s, n, H->h[ML].p, H->gy.p, H->part.p);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(MB), 0, s, np, MH * MO, H->part.p, grad + OFF_WOUT);
    hipLaunchKernelGGL(k_colsum3, dim3(np), dim3(MB), 0, s, n, H->gy.p, H->dpart.p);
    hipLaunchKernelGGL(k_colsum_out, dim3(1), dim3(64), 0, s, np, H->dpart.p, MO, grad + OFF_BOUT);
    for (int l = ML - 1; l >= 0; --l) {
        hipLaunchKernelGGL(k_mp_bwd1, dim3(vgrid((n + VB - 1) / VB)), dim3(MB), 4 * MH * MH * sizeof(float), s, n,
                           H->gp.p, P, l, H->gh.p,
                           H->a[l].p, H->ga.p, H->gmd.p, H->gd.p);
        hipLaunchKernelGGL((k_xty<MH, MH>), dim3(np), dim3(MB), 0, s, n, H->h[l].p, H->ga.p, H->part.p);
        hipLaunchKernelGGL(k_sum_parts, dim3(16), dim3(MB), 0, s, np, MH * MH, H->part.p, grad + off_ws(l));
        hipLaunchKernelGGL((k_xty<MH, MH>), dim3(np), dim3(MB), 0, s, n, H->m[l].p, H->ga.p, H->part.p);
        hipLaunchKernelGGL(k_sum_parts, dim3(16), dim3(MB), 0, s, np, MH * MH, H->part.p, grad + off_wn(l));
        hipLaunchKernelGGL((k_xty<MD, MH>), dim3(np), dim3(MB), 0, s, n, H->d[l].p, H->ga.p, H->part.p);
        hipLaunchKernelGGL(k_sum_parts, dim3(48), dim3(MB), 0, s, np, MD * MH, H->part.p, grad + off_wd(l));
        hipLaunchKernelGGL(k_colsum, dim3(np), dim3(MB), 0, s, n, H->ga.p, H->dpart.p);
        hipLaunchKernelGGL(k_layer_small, dim3(1), dim3(64), 0, s, np, H->dpart.p, H->g[l].p, P, l, grad, H->gg.p);
        hipLaunchKernelGGL(k_mp_bwd2, dim3(vg), dim3(MB), 0, s, n, H->gp.p, H->gi.p, H->xf.p, H->invdl.p, P, l,
                           H->ga.p, H->gmd.p, H->gd.p, H->gg.p, H->gh.p);
    }
    hipLaunchKernelGGL(k_relu_mask, dim3((unsigned)std::min<int64_t>((n * MH + MB - 1) / MB, 65536)), dim3(MB), 0, s,
                       n, H->h[0].p, H->gh.p, H->ga.p);
    hipLaunchKernelGGL((k_xty<MF, MH>), dim3(np), dim3(MB), 0, s, n, H->X.p, H->ga.p, H->part.p);
    hipLaunchKernelGGL(k_sum_parts, dim3(4), dim3(MB), 0, s, np, MF * MH, H->part.p, grad + OFF_WIN);
    hipLaunchKernelGGL(k_colsum, dim3(np), dim3(MB), 0, s, n, H->ga.p, H->dpart.p);
    hipLaunchKernelGGL(k_colsum_out, dim3(1), dim3(64), 0, s, np, H->dpart.p, MH, grad + OFF_BIN);
    TE_CHECK_HIP(hipGetLastError());
}

// Loss of the last forward against target (scaled displacement [N][3]) and
// gradients of every parameter into grad[NPARAM].
extern "C" int mpnn_backward(mpnn_handle *H, const float *P, const float *target, float *grad, double *loss,
                             hipStream_t s) {
    return guarded([&] {
        TE_REQUIRE(H && P && target && grad, TE_EINVAL, "bad argument");
        TE_REQUIRE(H->have_forward, TE_EINVAL, "mpnn_backward needs a preceding mpnn_forward");
        const int64_t n = H->n;
        const int np = nparts_for(n);
        hipLaunchKernelGGL(k_out, dim3(np), dim3(MB), 0, s, n, P, H->h[ML].p, H->mask.p, H->y.p, target, H->gy.p,
                           H->gh.p, H->dpart.p);
        TE_CHECK_HIP(hipGetLastError());
        std::vector<double> lp;
        download(lp, H->dpart.p, np, s);
        double L = 0.0;
        for (double v : lp) L += v;
        if (loss) *loss = L / double(3 * n);
        backward_tail(H, P, grad, s);
        return TE_OK;
    });
}

// Gradients of a loss given dL/dy of the last forward (float [N][3]).
extern "C" int mpnn_backward_from(mpnn_handle *H, const float *P, const float *gy, float *grad, hipStream_t s) {
    return guarded([&] {
        TE_REQUIRE(H && P && gy && grad, TE_EINVAL, "bad argument");
        TE_REQUIRE(H->have_forward, TE_EINVAL, "mpnn_backward_from needs a preceding mpnn_forward");
        hipLaunchKernelGGL(k_gy_to_gh, dim3(vgrid(H->n)), dim3(MB), 0, s, H->n, P, H->mask.p, gy, H->gy.p, H->gh.p);
        TE_CHECK_HIP(hipGetLastError());
        backward_tail(H, P, grad, s);
        return TE_OK;
    });
}

// Relative energy error of the energy-optimally scaled guess of the last
// forward: loss = 1 - c^2 / (a e) with u = S_U y (constrained DOFs zero),
// t = S_U target, a = (u, A u), c = (u, A t), e = (t, A t) (A = level-0
// operator of the AMG handle), and gy = dloss/dy =
// S_U keep (-2c/(a e) A t + 2c^2/(a^2 e) A u).  A zero guess: loss 1, gy 0.
// Uses the AMG handle's solve workspace.
extern "C" int mpnn_energy_grad(mpnn_handle *H, amg_handle *A, const float *target, float *gy, double *loss,
                                hipStream_t s) {
    return guarded([&] {
        TE_REQUIRE(H && A && target && gy, TE_EINVAL, "bad argument");
        TE_REQUIRE(H->have_forward, TE_EINVAL, "mpnn_energy_grad needs a preceding mpnn_forward");
        Level &L0 = A->L[0];
        TE_REQUIRE(L0.n == H->n, TE_EINVAL, "AMG and MPNN sizes differ");
        const int64_t n = H->n, nv = 3 * n;
        const unsigned g = (unsigned)std::min<int64_t>((nv + MB - 1) / MB, 65536);
        // natural-order u and u_t in the AMG's z / p buffers, storage order in t / u
        hipLaunchKernelGGL(k_energy_prep, dim3(g), dim3(MB), 0, s, n, H->y.p, target, H->mask.p, A->z.p, A->p.p);
        permute_gather(A->z.p, A->t.p, L0.perm.p, n, 3, 1, s);
        permute_gather(A->p.p, A->u.p, L0.perm.p, n, 3, 1, s);
        sell_apply<double>(L0.A, A->t.p, A->q.p, nullptr, 0, 1, s);   // A u
        sell_apply<double>(L0.A, A->u.p, A->r.p, nullptr, 0, 1, s);   // A u_t
        double *part = A->partials.p, *sums = A->sums.p;
        dot_partials(A->t.p, A->q.p, nv, 1, part, s);
        reduce_partials(part, dot_nblocks(nv), 1, sums, s);
        dot_partials(A->t.p, A->r.p, nv, 1, part, s);
        reduce_partials(part, dot_nblocks(nv), 1, sums + 1, s);
        dot_partials(A->u.p, A->r.p, nv, 1, part, s);
        reduce_partials(part, dot_nblocks(nv), 1, sums + 2, s);
        std::vector<double> v;
        download(v, sums, 3, s);
        const double aa = v[0], c = v[1], e = v[2];
        TE_REQUIRE(e > 0, TE_EINVAL, "target has no energy");
        double ca = 0.0, cb = 0.0, L = 1.0;
        if (aa > 0) {
            L = 1.0 - c * c / (aa * e);
            ca = -2.0 * c / (aa * e) * S_U;
            cb = 2.0 * c * c / (aa * aa * e) * S_U;
        }
        if (loss) *loss = L;
        permute_scatter(A->q.p, A->z.p, L0.perm.p, n, 3, 1, s);   // A u, natural
        permute_scatter(A->r.p, A->p.p, L0.perm.p, n, 3, 1, s);   // A u_t, natural
        hipLaunchKernelGGL(k_energy_gy, dim3(g), dim3(MB), 0, s, n, A->p.p, A->z.p, H->mask.p, ca, cb, gy);
        TE_CHECK_HIP(hipGetLastError());
        return TE_OK;
    });
}

extern "C" int mpnn_adam_step(int64_t n, float *p, const float *g, float *m, float *v, int32_t step, float lr,
                              float b1, float b2, float eps, hipStream_t s) {
    return guarded([&] {
        TE_REQUIRE(n > 0 && p && g && m && v && step >= 1, TE_EINVAL, "bad argument");
        const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
        const unsigned gr = (unsigned)std::min<int64_t>((n + MB - 1) / MB, 65536);
        hipLaunchKernelGGL(k_adam, dim3(gr), dim3(MB), 0, s, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
        TE_CHECK_HIP(hipGetLastError());
        return TE_OK;
    });
}

// u0 = S_U * y of the last forward (float64 [N][3])
extern "C" int mpnn_guess(mpnn_handle *H, double *u0, hipStream_t s) {
    return guarded([&] {
        TE_REQUIRE(H && u0 && H->have_forward, TE_EINVAL, "bad argument or no forward pass");
        const unsigned g = (unsigned)std::min<int64_t>((H->n * 3 + MB - 1) / MB, 65536);
        hipLaunchKernelGGL(k_guess, dim3(g), dim3(MB), 0, s, H->n, H->y.p, u0);
        TE_CHECK_HIP(hipGetLastError());
        return TE_OK;
    });
}
