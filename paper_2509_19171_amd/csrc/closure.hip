// Learned relaxation-time closure: MLP inference (FP32 MFMA), training
// kernels (forward, backward, deterministic weight-gradient sums, Adam),
// coarse graining of a fine simulation onto a coarse one of the same
// elements, training targets, and their C entry points.
//
// Parameter blob (float32): mean[6], std[6], W1[64][6], b1[64], W2[64][64],
// b2[64], W3[64][64], b3[64], w4[64], b4[1], dtau_max[1]. The trainable
// parameters are the contiguous range W1 .. b4.
#include <mutex>
#include <cmath>
#include <string>
#include <vector>

#include "kernels_impl.h"
#include "ops.h"

namespace sel {

namespace {

constexpr int NF = 6, NH = 64;
constexpr int OFF_MEAN = 0, OFF_STD = 6, OFF_W1 = 12, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH, OFF_W4 = OFF_B3 + NH,
              OFF_B4 = OFF_W4 + NH, OFF_DMAX = OFF_B4 + 1, BLOB = OFF_DMAX + 1;
constexpr int OFF_TRAIN = OFF_W1, NTRAIN = OFF_DMAX - OFF_W1;  // 8833

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

// tanh x = 1 - 2 / (exp(2x) + 1) with the hardware exp2 and reciprocal
// (absolute error about 1e-7; exp2 overflow gives the limits +-1)
__device__ __forceinline__ float tanh_fast(float x)
{
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // exp(2x) = 2^(2x / ln 2)
    return 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
}

__device__ __forceinline__ float guard_dtau(float d, float tau, float dmax)
{
    // fallback to the plain method (0) for non-finite or out-of-range values
    return (d == d && d >= 0.f && d <= dmax * tau) ? d : 0.f;
}

// W2 and W3 into LDS by a workgroup of 256 threads: every load of a thread is
// issued before its first LDS store, so the workgroup waits for one memory
// round trip instead of one per loop iteration.
__device__ __forceinline__ void stage_hidden(const float *__restrict__ P, float (*sW2)[NH + 1],
                                             float (*sW3)[NH + 1], int tid)
{
    constexpr int PER = NH * NH / 256;
    float a[PER], b[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        a[i] = P[OFF_W2 + tid + 256 * i];
        b[i] = P[OFF_W3 + tid + 256 * i];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = tid + 256 * i;
        sW2[q / NH][q % NH] = a[i];
        sW3[q / NH][q % NH] = b[i];
    }
}

// Work layout (floats): Xn[n][8], H1, H2, H3, D1, D2, D3 [n][64], Z[n], DZ[n],
// grad[NTRAIN], loss partials [nblk] and the loss, weight-gradient partials
// [nchunk][NTRAIN].
struct TrainWork {
    float *Xn, *H1, *H2, *H3, *D1, *D2, *D3, *Z, *DZ, *grad, *part, *wpart;
};


// ------------------------------------------------------------ inference --
// One workgroup of 4 wavefronts; each wavefront runs a tile of RW = 32 rows
// through 6 -> 64 -> 64 -> 64 -> 1 with v_mfma_f32_16x16x4f32 for the three
// hidden layers (A = activations, B = W^T, 2 x 4 output tiles of 16 x 16,
// activations re-laid out through LDS between layers). 71 KB of LDS, so two
// workgroups share a CU. Each wavefront's activation buffer is its own and a
// wavefront's LDS operations complete in order, so inside the row loop only
// compiler scheduling barriers separate the layers: the four wavefronts of a
// workgroup run independently.
constexpr int RW = 32;  // rows per wavefront
// inference grid: at most 1024 workgroups (four per CU, two resident at a
// time), each looping over its tiles, so that a workgroup stages the weights
// for many tiles (4096 workgroups took 1.3% longer on 1.4 M rows)
constexpr int64_t kInferMaxBlocks = 1024;
constexpr int RT = RW / 16;

// TRAIN: the forward pass of a training step on rows idx[s] of X (all rows
// when idx is null): the normalised inputs, the three hidden layers and z of
// sample s are stored in T for the back-propagation.
template <bool TRAIN>
__global__ void __launch_bounds__(256) k_mlp(const float *__restrict__ P, const float *__restrict__ X,
                                             const int32_t *__restrict__ idx, int64_t n, float tau,
                                             float *__restrict__ zout, float *__restrict__ dtau, TrainWork T)
{
    __shared__ float sW1[NH][9];
    __shared__ float sW2[NH][NH + 1];
    __shared__ float sW3[NH][NH + 1];
    __shared__ float sb1[NH], sb2[NH], sb3[NH], sw4[NH];
    __shared__ float sH[4][RW][NH + 1];
    __shared__ float smean[NF], sistd[NF];
    const int tid = threadIdx.x;
    const float b4 = P[OFF_B4], dmax = P[OFF_DMAX];
    {
        // all loads first (one round trip), then the LDS stores
        float w1v[2], bv[4] = {0.f, 0.f, 0.f, 0.f}, mv = 0.f, sv = 1.f;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int q = tid + 256 * i, r = q / 8, c = q % 8;
            w1v[i] = (c < NF) ? P[OFF_W1 + r * NF + c] : 0.f;
        }
        if (tid < NH) {
            bv[0] = P[OFF_B1 + tid];
            bv[1] = P[OFF_B2 + tid];
            bv[2] = P[OFF_B3 + tid];
            bv[3] = P[OFF_W4 + tid];
        }
        if (tid < NF) {
            mv = P[OFF_MEAN + tid];
            sv = P[OFF_STD + tid];
        }
        stage_hidden(P, sW2, sW3, tid);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int q = tid + 256 * i;
            sW1[q / 8][q % 8] = w1v[i];
        }
        if (tid < NH) {
            sb1[tid] = bv[0];
            sb2[tid] = bv[1];
            sb3[tid] = bv[2];
            sw4[tid] = bv[3];
        }
        if (tid < NF) {
            smean[tid] = mv;
            sistd[tid] = 1.f / sv;
        }
    }
    __syncthreads();
    const int w = tid / 64, l = tid % 64;
    const int li = l & 15, lk = l >> 4;
    for (int64_t base = (int64_t)blockIdx.x * (4 * RW); base < n; base += (int64_t)gridDim.x * (4 * RW)) {
        // normalised inputs, K padded to 8: lane l fills row l % RW, columns 4 (l / RW) .. +3
        {
            const int rr = l % RW, c0 = 4 * (l / RW);
            const int64_t r = base + w * RW + rr;
            const int64_t row = (TRAIN && idx && r < n) ? (int64_t)idx[r] : r;
#pragma unroll
            for (int c = c0; c < c0 + 4; ++c) {
                const float x = (c < NF && r < n) ? (X[row * NF + c] - smean[c]) * sistd[c] : 0.f;
                sH[w][rr][c] = x;
                if (TRAIN && r < n) T.Xn[r * 8 + c] = x;
            }
        }
        __builtin_amdgcn_wave_barrier();
        // training: the hidden layer just written to sH, stored row by row
        auto store_layer = [&](float *H) {
            if constexpr (TRAIN) {
                for (int q = l; q < RW * NH; q += 64) {
                    const int rr = q / NH, c = q - rr * NH;
                    const int64_t r = base + w * RW + rr;
                    if (r < n) H[r * NH + c] = sH[w][rr][c];
                }
            }
        };
        f4 acc[RT][4];
        // hidden layer 1 (K = 8)
#pragma unroll
        for (int ti = 0; ti < RT; ++ti)
#pragma unroll
            for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            float a[RT], b[4];
#pragma unroll
            for (int t = 0; t < RT; ++t) a[t] = sH[w][16 * t + li][4 * ks + lk];
#pragma unroll
            for (int t = 0; t < 4; ++t) b[t] = sW1[16 * t + li][4 * ks + lk];
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int ti = 0; ti < RT; ++ti)
#pragma unroll
            for (int tj = 0; tj < 4; ++tj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int col = 16 * tj + li;
                    sH[w][16 * ti + 4 * lk + q][col] = tanh_fast(acc[ti][tj][q] + sb1[col]);
                }
        __builtin_amdgcn_wave_barrier();
        store_layer(T.H1);
        // hidden layers 2 and 3 (K = 64)
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            const float(*Wl)[NH + 1] = layer == 0 ? sW2 : sW3;
            const float *bl = layer == 0 ? sb2 : sb3;
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = f4{0.f, 0.f, 0.f, 0.f};
            for (int ks = 0; ks < NH / 4; ++ks) {
                float a[RT], b[4];
#pragma unroll
                for (int t = 0; t < RT; ++t) a[t] = sH[w][16 * t + li][4 * ks + lk];
#pragma unroll
                for (int t = 0; t < 4; ++t) b[t] = Wl[16 * t + li][4 * ks + lk];
#pragma unroll
                for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 4; ++tj)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int col = 16 * tj + li;
                        sH[w][16 * ti + 4 * lk + q][col] = tanh_fast(acc[ti][tj][q] + bl[col]);
                    }
            __builtin_amdgcn_wave_barrier();
            store_layer(layer == 0 ? T.H2 : T.H3);
        }
        // output layer: two lanes per row, halves of the 64 products
        {
            const int rr = l % RW, h = l / RW;
            float z = 0.f;
#pragma unroll 8
            for (int c = 32 * h; c < 32 * h + 32; ++c) z += sH[w][rr][c] * sw4[c];
            z += __shfl_xor(z, 32);
            z += b4;
            const int64_t r = base + w * RW + rr;
            if (h == 0 && r < n) {
                if constexpr (TRAIN) T.Z[r] = z;
                if (zout) zout[r] = z;
                if (dtau) dtau[r] = guard_dtau(tau * softplusf(z), tau, dmax);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ------------------------------------------------------------- training --
// backward workgroups: one tile of 4 RW rows each, at most 4096
constexpr int64_t train_blocks(int64_t n)
{
    return (n + 4 * RW - 1) / (4 * RW) < 4096 ? (n + 4 * RW - 1) / (4 * RW) : 4096;
}

// The weight gradient sums over the samples in chunks (at least 64 samples,
// at most 1024 chunks), then over the chunks in order: the result does not
// depend on the launch, and every chunk is a short loop of its own.
constexpr int64_t wgrad_chunk(int64_t n) { return (n + 1023) / 1024 < 64 ? 64 : (n + 1023) / 1024; }
constexpr int64_t wgrad_chunks(int64_t n) { return (n + wgrad_chunk(n) - 1) / wgrad_chunk(n); }
// floats of training work memory for n rows (layout of carve_work)
constexpr int64_t work_floats(int64_t n)
{
    return (8 + 6 * (int64_t)NH + 2) * n + NTRAIN + train_blocks(n) + 1 + wgrad_chunks(n) * NTRAIN;
}

TrainWork carve_work(float *w, int64_t n)
{
    TrainWork t;
    t.Xn = w;
    t.H1 = t.Xn + 8 * n;
    t.H2 = t.H1 + NH * n;
    t.H3 = t.H2 + NH * n;
    t.D1 = t.H3 + NH * n;
    t.D2 = t.D1 + NH * n;
    t.D3 = t.D2 + NH * n;
    t.Z = t.D3 + NH * n;
    t.DZ = t.Z + n;
    t.grad = t.DZ + n;
    t.part = t.grad + NTRAIN;
    t.wpart = t.part + train_blocks(n) + 1;
    return t;
}

// Back-propagation of the mean squared error of softplus(z) against y, on
// the tiles of k_mlp (one tile of 4 RW rows per workgroup): the deltas of a
// layer are formed in the wavefront's LDS buffer, D_l = (D_{l+1} W_{l+1}) (1 -
// H_l^2) with v_mfma_f32_16x16x4f32 (A = deltas, B = W), and stored row by row.
// dz = (2/n) (softplus(z) - y) sigmoid(z); D3 = dz w4 (1 - H3^2). Lane l holds
// column l of the wavefront's activations, loaded before any delta is stored.
// One loss partial (sum of squared residuals) per workgroup.
__global__ void __launch_bounds__(256) k_train_bwd(const float *__restrict__ P, const float *__restrict__ y,
                                                   const int32_t *__restrict__ idx, int64_t n, TrainWork T)
{
    __shared__ float sW2[NH][NH + 1];
    __shared__ float sW3[NH][NH + 1];
    __shared__ float sw4[NH];
    __shared__ float sH[4][RW][NH + 1];
    __shared__ float sdz[4][RW];
    __shared__ float red[256];
    const float *__restrict__ H1 = T.H1;
    const float *__restrict__ H2 = T.H2;
    const float *__restrict__ H3 = T.H3;
    const float *__restrict__ Z = T.Z;
    float *__restrict__ D1 = T.D1;
    float *__restrict__ D2 = T.D2;
    float *__restrict__ D3 = T.D3;
    float *__restrict__ DZ = T.DZ;
    const int tid = threadIdx.x;
    {
        const float w4 = tid < NH ? P[OFF_W4 + tid] : 0.f;
        stage_hidden(P, sW2, sW3, tid);
        if (tid < NH) sw4[tid] = w4;
    }
    __syncthreads();
    const int w = tid / 64, l = tid % 64;
    const int li = l & 15, lk = l >> 4;
    const float two_n = 2.f / float(n);
    float r2 = 0.f;
    for (int64_t base = (int64_t)blockIdx.x * (4 * RW); base < n; base += (int64_t)gridDim.x * (4 * RW)) {
        const int64_t r0 = base + w * RW;  // the wavefront's first row
        float h1[RW], h2[RW], h3[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const bool ok = r0 + i < n;
            h1[i] = ok ? H1[(r0 + i) * NH + l] : 0.f;
            h2[i] = ok ? H2[(r0 + i) * NH + l] : 0.f;
            h3[i] = ok ? H3[(r0 + i) * NH + l] : 0.f;
        }
        // residual and dz of the wavefront's rows
        if (l < RW) {
            const int64_t r = r0 + l;
            float dz = 0.f;
            if (r < n) {
                const float z = Z[r];
                const float res = softplusf(z) - y[idx ? (int64_t)idx[r] : r];
                r2 += res * res;
                dz = two_n * res / (1.f + expf(-z));
                DZ[r] = dz;
            }
            sdz[w][l] = dz;
        }
        __builtin_amdgcn_wave_barrier();
        // D3 = dz w4 (1 - H3^2)
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const float d = sdz[w][i] * sw4[l] * (1.f - h3[i] * h3[i]);
            if (r0 + i < n) D3[(r0 + i) * NH + l] = d;
            sH[w][i][l] = d;
        }
        __builtin_amdgcn_wave_barrier();
        // D2 from D3 through W3, then D1 from D2 through W2
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            const float(*Wl)[NH + 1] = layer == 0 ? sW3 : sW2;
            float *__restrict__ D = layer == 0 ? D2 : D1;
            f4 acc[RT][4];
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = f4{0.f, 0.f, 0.f, 0.f};
            for (int ks = 0; ks < NH / 4; ++ks) {
                float a[RT], b[4];
#pragma unroll
                for (int t = 0; t < RT; ++t) a[t] = sH[w][16 * t + li][4 * ks + lk];
#pragma unroll
                for (int t = 0; t < 4; ++t) b[t] = Wl[4 * ks + lk][16 * t + li];
#pragma unroll
                for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 4; ++tj)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) sH[w][16 * ti + 4 * lk + q][16 * tj + li] = acc[ti][tj][q];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int i = 0; i < RW; ++i) {
                const float h = layer == 0 ? h2[i] : h1[i];
                const float d = sH[w][i][l] * (1.f - h * h);
                if (r0 + i < n) D[(r0 + i) * NH + l] = d;
                sH[w][i][l] = d;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    red[tid] = r2;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) T.part[blockIdx.x] = red[0];
}

// Partial gradients of one chunk of samples per workgroup. The weight blocks
// G_l[m][k] = sum_s D_l[s][m] A_{l-1}[s][k] of W1 (inputs padded to 8
// columns), W2 and W3 run on v_mfma_f32_16x16x4f32 with A = D^T and B =
// A_{l-1}, wavefront w taking the output rows 16 w .. 16 w + 15; the biases,
// w4 and b4 are plain sums in sample order.
__global__ void __launch_bounds__(256) k_train_wgrad(int64_t n, int64_t chunk, TrainWork T)
{
    const int64_t s0 = (int64_t)blockIdx.x * chunk;
    const int64_t s1 = s0 + chunk < n ? s0 + chunk : n;
    const float *__restrict__ Xn = T.Xn;
    const float *__restrict__ H1 = T.H1;
    const float *__restrict__ H2 = T.H2;
    const float *__restrict__ H3 = T.H3;
    const float *__restrict__ D1 = T.D1;
    const float *__restrict__ D2 = T.D2;
    const float *__restrict__ D3 = T.D3;
    const float *__restrict__ DZ = T.DZ;
    float *__restrict__ out = T.wpart + (int64_t)blockIdx.x * NTRAIN;
    const int tid = threadIdx.x, w = tid / 64, l = tid % 64;
    const int li = l & 15, lk = l >> 4;
    const int m = 16 * w + li;  // the output row this lane feeds as A
    f4 g1 = {0.f, 0.f, 0.f, 0.f}, g2[4], g3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) g2[t] = g3[t] = f4{0.f, 0.f, 0.f, 0.f};
    for (int64_t s = s0; s < s1; s += 4) {
        const int64_t sr = s + lk;
        const bool ok = sr < s1;
        const float a1 = ok ? D1[sr * NH + m] : 0.f;
        const float a2 = ok ? D2[sr * NH + m] : 0.f;
        const float a3 = ok ? D3[sr * NH + m] : 0.f;
        const float b1 = (ok && li < 8) ? Xn[sr * 8 + li] : 0.f;
        float b2[4], b3[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            b2[t] = ok ? H1[sr * NH + 16 * t + li] : 0.f;
            b3[t] = ok ? H2[sr * NH + 16 * t + li] : 0.f;
        }
        g1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, g1, 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            g2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2[t], g2[t], 0, 0, 0);
            g3[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, b3[t], g3[t], 0, 0, 0);
        }
    }
    // output (row 16 w + 4 lk + q, column 16 t + li) of each accumulator
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = 16 * w + 4 * lk + q;
        if (li < NF) out[OFF_W1 - OFF_TRAIN + row * NF + li] = g1[q];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            out[OFF_W2 - OFF_TRAIN + row * NH + 16 * t + li] = g2[t][q];
            out[OFF_W3 - OFF_TRAIN + row * NH + 16 * t + li] = g3[t][q];
        }
    }
    // b1, b2, b3 (one thread per entry), w4 (one per weight) and b4
    {
        const int k = tid % NH;
        const float *__restrict__ D = tid < 64 ? D1 : tid < 128 ? D2 : D3;
        float g = 0.f, gb = 0.f;
        if (tid < 192) {
#pragma unroll 16
            for (int64_t s = s0; s < s1; ++s) g += D[s * NH + k];
        } else {
#pragma unroll 16
            for (int64_t s = s0; s < s1; ++s) {
                const float dz = DZ[s];
                g += dz * H3[s * NH + k];
                gb += dz;
            }
        }
        const int off = tid < 64 ? OFF_B1 : tid < 128 ? OFF_B2 : tid < 192 ? OFF_B3 : OFF_W4;
        out[off - OFF_TRAIN + k] = g;
        if (tid == 192) out[OFF_B4 - OFF_TRAIN] = gb;
    }
}

// the gradient: the partials summed in chunk order; the thread after the
// last parameter sums the nb loss partials of the backward pass into *loss
__global__ void __launch_bounds__(256) k_train_wsum(int64_t nchunk, int nb, int64_t n, TrainWork T, float *loss)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == NTRAIN) {
        const float *__restrict__ part = T.part;
        float s = 0.f;
#pragma unroll 16
        for (int b = 0; b < nb; ++b) s += part[b];
        loss[0] = s / float(n);
    }
    if (q >= NTRAIN) return;
    const float *__restrict__ wp = T.wpart;
    float g = 0.f;
#pragma unroll 16
    for (int64_t c = 0; c < nchunk; ++c) g += wp[c * NTRAIN + q];
    T.grad[q] = g;
}

// forward, back-propagation, loss and gradient of n samples into T
void launch_gradient(const float *P, const float *X, const float *y, const int32_t *idx, int64_t n, TrainWork T,
                     float *dloss, hipStream_t st)
{
    int64_t nbf = (n + 4 * RW - 1) / (4 * RW);
    if (nbf > 4096) nbf = 4096;
    hipLaunchKernelGGL(k_mlp<true>, dim3((unsigned)nbf), dim3(256), 0, st, P, X, idx, n, 1.f, nullptr, nullptr, T);
    // one loss partial per backward workgroup
    const int64_t nbb = train_blocks(n);
    hipLaunchKernelGGL(k_train_bwd, dim3((unsigned)nbb), dim3(256), 0, st, P, y, idx, n, T);
    const int64_t nchunk = wgrad_chunks(n);  // at most 1024
    hipLaunchKernelGGL(k_train_wgrad, dim3((unsigned)nchunk), dim3(256), 0, st, n, wgrad_chunk(n), T);
    hipLaunchKernelGGL(k_train_wsum, dim3((NTRAIN + 1 + 255) / 256), dim3(256), 0, st, nchunk, (int)nbb, n, T,
                       dloss);
}

// Adam (Kingma & Ba), bias-corrected, on the trainable range
__global__ void k_adam(float *P, float *m, float *v, const float *g, int64_t t, float lr, float b1, float b2, float eps)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NTRAIN) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.f - powf(b1, float(t)));
    const float vh = vq / (1.f - powf(b2, float(t)));
    P[OFF_TRAIN + q] -= lr * mh / (sqrtf(vh) + eps);
}

// --------------------------------------------------------- coarse graining --
// One workgroup per element, one thread per fine node; the projection matrix
// Pm[ic][jf] is applied along r, s (and t) through LDS (sizes change per pass).
template <int DIM, int Q, typename T, bool DEV>
__global__ void k_coarse(NodeMap Mf, const T *ff, NodeMap Mc, T *fc, const double *Pm, int nf1, int nc1, double rho0)
{
    __shared__ double b0[1024], b1[1024];
    __shared__ double sP[kMaxN1 * kMaxN1];
    const int64_t e = blockIdx.x;
    const int p = threadIdx.x;
    const int npf = blockDim.x;
    for (int q = p; q < nc1 * nf1; q += npf) sP[q] = Pm[q];
    const int i = p % nf1, j = (p / nf1) % nf1, k = (DIM == 3) ? p / (nf1 * nf1) : 0;
    bool ownf;
    const SIdx sf = Mf.sidx(e, p, ownf);
    bool ownc = false;
    SIdx sc{0, 0};
    const bool on_coarse = i < nc1 && j < nc1 && (DIM == 2 || k < nc1);
    if (on_coarse) sc = Mc.sidx(e, i + nc1 * j + (DIM == 3 ? nc1 * nc1 * k : 0), ownc);
    for (int a = 0; a < Q; ++a) {
        b0[p] = double(ff[sf.base + (int64_t)a * sf.stride]);
        __syncthreads();
        if (i < nc1) {  // along r: [nc1][nf1][nf1]
            double v = 0.0;
            for (int c = 0; c < nf1; ++c) v += sP[i * nf1 + c] * b0[c + nf1 * j + nf1 * nf1 * k];
            b1[i + nc1 * j + nc1 * nf1 * k] = v;
        }
        __syncthreads();
        double v = 0.0;
        if (i < nc1 && j < nc1) {  // along s: [nc1][nc1][nf1]
            for (int c = 0; c < nf1; ++c) v += sP[j * nf1 + c] * b1[i + nc1 * c + nc1 * nf1 * k];
        }
        if (DIM == 3) {
            __syncthreads();
            if (i < nc1 && j < nc1) b0[i + nc1 * j + nc1 * nc1 * k] = v;
            __syncthreads();
            if (on_coarse) {
                v = 0.0;
                for (int c = 0; c < nf1; ++c) v += sP[k * nf1 + c] * b0[i + nc1 * j + nc1 * nc1 * c];
            }
        }
        if (on_coarse && ownc) fc[sc.base + (int64_t)a * sc.stride] = T(v);
        __syncthreads();
    }
    (void)rho0;
}

// Training target per coarse element: P(u), P(u u) from the fine state,
// S-bar from P(u) with the coarse metric, tau_sgs = P(uu) - P(u) P(u),
// nu_t = max(0, -<dev tau_sgs : S-bar> / <2 S-bar : S-bar>), dtau* = nu_t / (c_s^2 dt),
// written as y = dtau* / tau (the target of softplus(z)) on every coarse node.
template <int DIM, int Q, typename T, bool DEV>
__global__ void k_targets(NodeMap Mf, const T *ff, const double *Pm, int nf1, int nc1, const T *Gmc,
                          const double *wJc, const double *Dc, double rho0, double dtc, double tauc, float *y)
{
    constexpr int NFLD = DIM + DIM * (DIM + 1) / 2;
    __shared__ double b0[1024], b1[1024];
    __shared__ double sP[kMaxN1 * kMaxN1];
    __shared__ double cf[NFLD][512];
    const int64_t e = blockIdx.x;
    const int p = threadIdx.x;
    const int npf = blockDim.x;
    const int ncp = (DIM == 3) ? nc1 * nc1 * nc1 : nc1 * nc1;
    for (int q = p; q < nc1 * nf1; q += npf) sP[q] = Pm[q];
    const int i = p % nf1, j = (p / nf1) % nf1, k = (DIM == 3) ? p / (nf1 * nf1) : 0;
    bool own;
    const SIdx sf = Mf.sidx(e, p, own);
    double m = 0, jv[3] = {0, 0, 0};
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        const double v = double(ff[sf.base + (int64_t)a * sf.stride]);
        m += v;
        if constexpr (lat_e<DIM, Q>(a, 0) != 0) jv[0] += lat_e<DIM, Q>(a, 0) * v;
        if constexpr (lat_e<DIM, Q>(a, 1) != 0) jv[1] += lat_e<DIM, Q>(a, 1) * v;
        if constexpr (lat_e<DIM, Q>(a, 2) != 0) jv[2] += lat_e<DIM, Q>(a, 2) * v;
    });
    const double rho = DEV ? rho0 + m : m;
    double fld[NFLD];
    for (int c = 0; c < DIM; ++c) fld[c] = jv[c] / rho;
    {
        int q = DIM;
        for (int r = 0; r < DIM; ++r)
            for (int c = r; c < DIM; ++c) fld[q++] = fld[r] * fld[c];
    }
    const bool on_coarse = i < nc1 && j < nc1 && (DIM == 2 || k < nc1);
    const int pc = i + nc1 * j + (DIM == 3 ? nc1 * nc1 * k : 0);
    for (int q = 0; q < NFLD; ++q) {
        b0[p] = fld[q];
        __syncthreads();
        if (i < nc1) {
            double v = 0.0;
            for (int c = 0; c < nf1; ++c) v += sP[i * nf1 + c] * b0[c + nf1 * j + nf1 * nf1 * k];
            b1[i + nc1 * j + nc1 * nf1 * k] = v;
        }
        __syncthreads();
        double v = 0.0;
        if (i < nc1 && j < nc1)
            for (int c = 0; c < nf1; ++c) v += sP[j * nf1 + c] * b1[i + nc1 * c + nc1 * nf1 * k];
        if (DIM == 3) {
            __syncthreads();
            if (i < nc1 && j < nc1) b0[i + nc1 * j + nc1 * nc1 * k] = v;
            __syncthreads();
            if (on_coarse) {
                v = 0.0;
                for (int c = 0; c < nf1; ++c) v += sP[k * nf1 + c] * b0[i + nc1 * j + nc1 * nc1 * c];
            }
        }
        if (on_coarse) cf[q][pc] = v;
        __syncthreads();
    }
    double num = 0.0, den = 0.0;
    if (on_coarse) {
        const int idx[3] = {i, j, k};
        const int str[3] = {1, nc1, nc1 * nc1};
        double du[3][3] = {};
        for (int mm = 0; mm < DIM; ++mm) {
            const int b = pc - idx[mm] * str[mm];
            for (int c = 0; c < nc1; ++c) {
                const double dq = Dc[idx[mm] * nc1 + c];
                for (int q = 0; q < DIM; ++q) du[q][mm] += dq * cf[q][b + c * str[mm]];
            }
        }
        const double wj = wJc[e * ncp + pc];
        double A[3][3] = {};
        for (int mm = 0; mm < DIM; ++mm)
            for (int q = 0; q < DIM; ++q) {
                const double drdx = double(Gmc[(e * DIM * DIM + mm * DIM + q) * ncp + pc]) / wj;
                for (int c = 0; c < DIM; ++c) A[c][q] += du[c][mm] * drdx;
            }
        double S[3][3] = {}, tau[3][3] = {};
        int q = DIM;
        for (int r = 0; r < DIM; ++r)
            for (int c = r; c < DIM; ++c) {
                tau[r][c] = tau[c][r] = cf[q][pc] - cf[r][pc] * cf[c][pc];
                ++q;
            }
        double tr = 0.0;
        for (int r = 0; r < DIM; ++r) tr += tau[r][r];
        for (int r = 0; r < DIM; ++r)
            for (int c = 0; c < DIM; ++c) {
                S[r][c] = 0.5 * (A[r][c] + A[c][r]);
                const double td = tau[r][c] - (r == c ? tr / DIM : 0.0);
                num += wj * td * S[r][c];
                den += wj * 2.0 * S[r][c] * S[r][c];
            }
    }
    b0[p] = num;  // b0 and b1 are free after the last pass
    b1[p] = den;
    __syncthreads();
    if (p == 0) {
        double sn = 0.0, sd = 0.0;
        for (int q = 0; q < npf; ++q) {
            sn += b0[q];
            sd += b1[q];
        }
        const double nut = (sd > 0.0) ? fmax(0.0, -sn / sd) : 0.0;
        b0[0] = nut / (dtc / 3.0) / tauc;
    }
    __syncthreads();
    if (p < ncp) y[e * ncp + p] = float(b0[0]);
}

template <int DIM, int Q, typename T, bool DEV>
NodeMap nodemap_of(const sel_sim *s)
{
    NodeMap M;
    M.pcode = s->pcode;
    M.bmap = s->bmap;
    M.bown = s->bown;
    M.E = s->E;
    M.Gi = s->Gi;
    M.QGi = (int64_t)Q * s->Gi;
    M.NP = s->np;
    M.NI = s->nint;
    M.NB = s->nbe;
    M.Q = Q;
    return M;
}

template <int DIM, int Q, typename T, bool DEV>
int run_coarse(const sel_sim *f, sel_sim *c, const double *dP, bool targets, float *y)
{
    const dim3 grid((unsigned)f->E), block((unsigned)f->np);
    if (!targets) {
        hipLaunchKernelGGL((k_coarse<DIM, Q, T, DEV>), grid, block, 0, c->stream, nodemap_of<DIM, Q, T, DEV>(f),
                           static_cast<const T *>(f->f[f->cur]), nodemap_of<DIM, Q, T, DEV>(c),
                           static_cast<T *>(c->f[c->cur]), dP, f->n1, c->n1, f->p.rho0);
    } else {
        hipLaunchKernelGGL((k_targets<DIM, Q, T, DEV>), grid, block, 0, c->stream, nodemap_of<DIM, Q, T, DEV>(f),
                           static_cast<const T *>(f->f[f->cur]), dP, f->n1, c->n1, static_cast<const T *>(c->Gm),
                           c->wJ, c->geoD, f->p.rho0, c->p.dt, c->tau, y);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("coarse-graining launch failed: ") + hipGetErrorString(err));
        return SEL_EDEVICE;
    }
    return SEL_OK;
}

int coarse_dispatch(const sel_sim *f, sel_sim *c, const double *dP, bool targets, float *y)
{
    const bool f32 = f->prec == SEL_FP32_DEV;
    if (f->dim == 2 && f->Q == 9)
        return f32 ? run_coarse<2, 9, float, true>(f, c, dP, targets, y) : run_coarse<2, 9, double, false>(f, c, dP, targets, y);
    if (f->dim == 3 && f->Q == 27)
        return f32 ? run_coarse<3, 27, float, true>(f, c, dP, targets, y)
                   : run_coarse<3, 27, double, false>(f, c, dP, targets, y);
    if (f->dim == 3 && f->Q == 19)
        return f32 ? run_coarse<3, 19, float, true>(f, c, dP, targets, y)
                   : run_coarse<3, 19, double, false>(f, c, dP, targets, y);
    set_error("coarse graining: unsupported lattice");
    return SEL_EUNSUPPORTED;
}

int check_pair(const sel_sim *f, const sel_sim *c)
{
    if (!f || !c) {
        set_error("coarse graining: null simulation");
        return SEL_EINVAL;
    }
    if (f->dim != c->dim || f->Q != c->Q || f->prec != c->prec || f->E != c->E || c->N > f->N) {
        set_error("coarse graining: simulations must share dim, lattice, storage and elements, coarse N <= fine N");
        return SEL_EINVAL;
    }
    if (f->np > 1024 || c->np > 512) {
        set_error("coarse graining: order too high (fine np <= 1024, coarse np <= 512)");
        return SEL_EUNSUPPORTED;
    }
    return SEL_OK;
}

}  // namespace

int launch_mlp_infer(sel_sim *s)
{
    const int64_t n = s->Gtot;
    int64_t nb = (n + 4 * RW - 1) / (4 * RW);
    if (nb > kInferMaxBlocks) nb = kInferMaxBlocks;
    hipLaunchKernelGGL(k_mlp<false>, dim3((unsigned)nb), dim3(256), 0, s->stream, s->cl_params, s->cl_X, nullptr, n,
                       float(s->tau), nullptr, s->cl_dtau, TrainWork{});
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("closure inference launch failed: ") + hipGetErrorString(err));
        return SEL_EDEVICE;
    }
    return SEL_OK;
}

}  // namespace sel

using sel::set_error;

extern "C" int64_t sel_closure_len(void) { return sel::BLOB; }

extern "C" int sel_closure_set(sel_sim *s, const float *params, int64_t len)
{
    if (!s) {
        set_error("sel_closure_set: null sim");
        return SEL_EINVAL;
    }
    if (!params) {
        s->closure_on = false;
        return SEL_OK;
    }
    if (!s->closure_space) {
        set_error("sel_closure_set: the simulation was created without closure buffers (pass a blob to sel_init)");
        return SEL_ESTATE;
    }
    if (len != sel::BLOB) {
        set_error("sel_closure_set: blob length must be sel_closure_len()");
        return SEL_EINVAL;
    }
    if (hipMemcpyAsync(s->cl_params, params, sizeof(float) * len, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess) {
        set_error("sel_closure_set: upload failed");
        return SEL_EDEVICE;
    }
    s->closure_on = true;
    return SEL_OK;
}

extern "C" int sel_closure_features(sel_sim *s, float *d_X)
{
    if (!s || !d_X) {
        set_error("sel_closure_features: null argument");
        return SEL_EINVAL;
    }
    return sel::find_ops(s->dim, s->N, s->Q, s->prec)->features(s, d_X, 0, 0);
}

extern "C" int sel_closure_dtau(sel_sim *s, float *d_dtau)
{
    if (!s || !d_dtau) {
        set_error("sel_closure_dtau: null argument");
        return SEL_EINVAL;
    }
    if (!s->closure_on) {
        set_error("sel_closure_dtau: no closure attached");
        return SEL_ESTATE;
    }
    if (int rc = sel::find_ops(s->dim, s->N, s->Q, s->prec)->features(s, s->cl_X, 1, 0)) return rc;
    if (int rc = sel::launch_mlp_infer(s)) return rc;
    if (hipMemcpyAsync(d_dtau, s->cl_dtau, sizeof(float) * s->Gtot, hipMemcpyDeviceToDevice, s->stream) != hipSuccess) {
        set_error("sel_closure_dtau: copy failed");
        return SEL_EDEVICE;
    }
    return SEL_OK;
}

static int projection_on_device(const sel_sim *f, const sel_sim *c, double **dP)
{
    std::vector<double> Pm((size_t)c->n1 * f->n1);
    if (sel::build_projection(f->N, c->N, Pm.data())) {
        set_error("coarse graining: projection table");
        return SEL_EINVAL;
    }
    if (hipMalloc(dP, sizeof(double) * Pm.size()) != hipSuccess) {
        set_error("coarse graining: allocation failed");
        return SEL_ENOMEM;
    }
    if (hipMemcpyAsync(*dP, Pm.data(), sizeof(double) * Pm.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipFree(*dP);
        set_error("coarse graining: upload failed");
        return SEL_EDEVICE;
    }
    return SEL_OK;
}

extern "C" int sel_coarse_grain(const sel_sim *fine, sel_sim *coarse)
{
    if (int rc = sel::check_pair(fine, coarse)) return rc;
    double *dP = nullptr;
    if (int rc = projection_on_device(fine, coarse, &dP)) return rc;
    int rc = hipStreamSynchronize(fine->stream) == hipSuccess ? SEL_OK : SEL_EDEVICE;
    if (!rc) rc = sel::coarse_dispatch(fine, coarse, dP, false, nullptr);
    if (!rc && hipStreamSynchronize(coarse->stream) != hipSuccess) rc = SEL_EDEVICE;
    (void)hipFree(dP);
    return rc;
}

extern "C" int sel_closure_targets(const sel_sim *fine, sel_sim *coarse, float *d_y)
{
    if (!d_y) {
        set_error("sel_closure_targets: null output");
        return SEL_EINVAL;
    }
    if (int rc = sel::check_pair(fine, coarse)) return rc;
    double *dP = nullptr;
    if (int rc = projection_on_device(fine, coarse, &dP)) return rc;
    int rc = hipStreamSynchronize(fine->stream) == hipSuccess ? SEL_OK : SEL_EDEVICE;
    if (!rc) rc = sel::coarse_dispatch(fine, coarse, dP, true, d_y);
    if (!rc && hipStreamSynchronize(coarse->stream) != hipSuccess) rc = SEL_EDEVICE;
    (void)hipFree(dP);
    return rc;
}

extern "C" int sel_mlp_forward(const float *d_params, const float *d_X, int64_t n, double tau, float *d_z,
                               float *d_dtau, void *stream)
{
    if (!d_params || !d_X || n < 0) {
        set_error("sel_mlp_forward: bad argument");
        return SEL_EINVAL;
    }
    if (n == 0) return SEL_OK;
    int64_t nb = (n + 4 * sel::RW - 1) / (4 * sel::RW);
    if (nb > sel::kInferMaxBlocks) nb = sel::kInferMaxBlocks;
    hipLaunchKernelGGL(sel::k_mlp<false>, dim3((unsigned)nb), dim3(256), 0, static_cast<hipStream_t>(stream), d_params,
                       d_X, nullptr, n, float(tau), d_z, d_dtau, sel::TrainWork{});
    if (hipGetLastError() != hipSuccess) {
        set_error("sel_mlp_forward: launch failed");
        return SEL_EDEVICE;
    }
    return SEL_OK;
}

extern "C" int64_t sel_mlp_work_floats(int64_t n) { return sel::work_floats(n); }

// one Adam step with the training work memory at d_work (both entry points)
static int train_step(const char *who, float *d_params, float *d_m, float *d_v, const float *d_X, const float *d_y,
                      const int32_t *d_idx, int64_t n, int64_t t, double lr, double b1, double b2, double eps,
                      float *d_work, double *loss, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    sel::TrainWork T = sel::carve_work(d_work, n);
    float *dloss = T.part + sel::train_blocks(n);
    sel::launch_gradient(d_params, d_X, d_y, d_idx, n, T, dloss, st);
    const unsigned gq = (sel::NTRAIN + 255) / 256;
    hipLaunchKernelGGL(sel::k_adam, dim3(gq), dim3(256), 0, st, d_params, d_m, d_v, T.grad, t, float(lr), float(b1),
                       float(b2), float(eps));
    if (hipGetLastError() != hipSuccess) {
        set_error(std::string(who) + ": launch failed");
        return SEL_EDEVICE;
    }
    if (loss) {
        float h = 0.f;
        if (hipMemcpyAsync(&h, dloss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error(std::string(who) + ": device error");
            return SEL_EDEVICE;
        }
        *loss = h;
    }
    return SEL_OK;
}

extern "C" int sel_mlp_train_step(float *d_params, float *d_m, float *d_v, const float *d_X, const float *d_y,
                                  const int32_t *d_idx, int64_t n, int64_t t, double lr, double b1, double b2, double eps, float *d_work,
                                  double *loss, void *stream)
{
    if (!d_params || !d_m || !d_v || !d_X || !d_y || !d_work || n < 1 || t < 1) {
        set_error("sel_mlp_train_step: bad argument");
        return SEL_EINVAL;
    }
    return train_step("sel_mlp_train_step", d_params, d_m, d_v, d_X, d_y, d_idx, n, t, lr, b1, b2, eps, d_work, loss,
                      stream);
}

// ------------------------------------------------ allocation-free training --
// The training work memory of sel_mlp_train_step_noalloc: one file-scope
// device array (each GPU the library runs on holds its own copy until the
// process ends). Host code never passes the array's name to a kernel (on the
// host it only stands for the symbol): the device address is looked up once
// per device with hipGetSymbolAddress, on the first call made with that
// device current, and kept per device. Every call writes each value of the
// work memory it later reads (forward activations, deltas, chunk partials,
// gradient, loss), so nothing needs clearing between calls.
constexpr int64_t kNoAllocRows = 4096;
constexpr int64_t kNoAllocFloats = sel::work_floats(kNoAllocRows);
static __device__ __align__(256) float scratch[kNoAllocFloats];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[kMaxDevices] = {};

static int scratch_of_current_device(float **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("sel_mlp_train_step_noalloc: no usable current device");
        return SEL_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("sel_mlp_train_step_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
            return SEL_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SEL_OK;
}

extern "C" int sel_mlp_train_step_noalloc(float *d_params, float *d_m, float *d_v, const float *d_X,
                                          const float *d_y, const int32_t *d_idx, int64_t n, int64_t t, double lr,
                                          double b1, double b2, double eps, double *loss, void *stream)
{
    if (!d_params || !d_m || !d_v || !d_X || !d_y || n < 1 || t < 1) {
        set_error("sel_mlp_train_step_noalloc: bad argument");
        return SEL_EINVAL;
    }
    if (n > kNoAllocRows) {
        set_error("sel_mlp_train_step_noalloc: at most 4096 rows per call (its fixed work memory); use "
                  "sel_mlp_train_step with a work buffer for larger minibatches");
        return SEL_EINVAL;
    }
    float *work = nullptr;
    if (int rc = scratch_of_current_device(&work)) return rc;
    return train_step("sel_mlp_train_step_noalloc", d_params, d_m, d_v, d_X, d_y, d_idx, n, t, lr, b1, b2, eps, work,
                      loss, stream);
}

extern "C" int sel_mlp_gradient(const float *d_params, const float *d_X, const float *d_y, const int32_t *d_idx,
                                int64_t n, float *d_work, float *d_grad, double *loss, void *stream)
{
    if (!d_params || !d_X || !d_y || !d_work || !d_grad || n < 1) {
        set_error("sel_mlp_gradient: bad argument");
        return SEL_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    sel::TrainWork T = sel::carve_work(d_work, n);
    float *dloss = T.part + sel::train_blocks(n);
    sel::launch_gradient(d_params, d_X, d_y, d_idx, n, T, dloss, st);
    if (hipMemcpyAsync(d_grad, T.grad, sizeof(float) * sel::NTRAIN, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        set_error("sel_mlp_gradient: copy failed");
        return SEL_EDEVICE;
    }
    if (loss) {
        float h = 0.f;
        if (hipMemcpyAsync(&h, dloss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("sel_mlp_gradient: device error");
            return SEL_EDEVICE;
        }
        *loss = h;
    }
    return SEL_OK;
}
