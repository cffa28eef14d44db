// Learned DOS reconstruction: a small multilayer perceptron trained and run
// with hand-written kernels (BF16 matrix-core GEMMs with FP32 accumulation,
// FP32 master weights and Adam).
//
//   x (n_in) -> h1 = gelu(x W1 + b1) -> h2 = gelu(h1 W2 + b2)
//            -> h3 = gelu(h2 W3 + b3) -> z = h3 W4 + b4, s = h3 w5 + b5
//   q = softmax(z)   (DOS mass per energy bin)      e = softplus(s)   (predicted L1 error)
//   loss = (1/B) sum_b [ -sum_k p_bk log q_bk + lam (e_b - t_b)^2 ]
//
// GELU is the exact x Phi(x).  The error head is folded into the last GEMM
// as one extra output column (W4ext = [W4 | w5 | 0]).  All GEMM operands are
// BF16 (weights are BF16 copies of the FP32 masters, activations are rounded
// to BF16 when they are stored); products accumulate in FP32 on the MFMA
// units; pre-activations, logits and gradients of the biases stay in FP32.
//
// Internal parameter layout (FP32 masters, gradients and Adam moments share
// it): W1p [K1p x H] (rows n_in .. K1p-1 zero), b1 [H], W2 [H x H], b2 [H],
// W3 [H x H], b3 [H], W4ext [H x N4p], b4ext [N4p], with K1p = n_in rounded
// up to 32 and N4p = n_out + 1 rounded up to 16.  Padding entries have zero
// gradients, so they stay zero under Adam.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kpm_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace kpm {
namespace mlp {
namespace {

// float -> bf16 bits, round to nearest even (inputs are finite)
__device__ inline unsigned short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<unsigned short>(u >> 16);
}

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS = 2, EPI_DGELU = 3 };

constexpr int kTile = 64;    // C tile per workgroup (64 x 64), 4 waves of 32 x 32
constexpr int kKStep = 32;   // K per MFMA 16x16x32
constexpr int kLdsK = 40;    // LDS row pitch in bf16 (80 bytes: rows start on distinct banks)

// C[M x N] = op(A)[M x K] op(B)[K x N] with BF16 operands (bits in
// unsigned short) and FP32 accumulation.  op(A)(i, k) = TA ? A[k*lda + i] :
// A[i*lda + k]; op(B)(k, j) = TB ? B[j*ldb + k] : B[k*ldb + j].
// Epilogue per element (i, j) of C:
//   EPI_STORE      c32[i*ldc + j] = acc
//   EPI_BIAS_GELU  a = acc + bias[j]; c32 = a; c16[i*ldc + j] = bf16(gelu(a))
//   EPI_BIAS       c32 = acc + bias[j]
//   EPI_DGELU      d = acc * gelu'(aux[i*ldc + j]); c32 = d; c16 = bf16(d)
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256)
gemm_kernel(const unsigned short* __restrict__ A, const unsigned short* __restrict__ B, int M, int N, int K,
            int lda, int ldb, int ldc, const float* __restrict__ bias, const float* __restrict__ aux,
            float* __restrict__ c32, unsigned short* __restrict__ c16) {
    __shared__ __attribute__((aligned(16))) unsigned short As[kTile][kLdsK];   // [i][k]
    __shared__ __attribute__((aligned(16))) unsigned short Bs[kTile][kLdsK];   // [j][k]
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int wr = wave >> 1, wc = wave & 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += kKStep) {
        // A tile: 64 x 32 elements, 8 per thread
        if (!TA) {
            const int i = t >> 2, kc = (t & 3) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gi = m0 + i, gk = k0 + kc + e;
                As[i][kc + e] = (gi < M && gk < K) ? A[static_cast<int64_t>(gi) * lda + gk] : 0;
            }
        } else {
            const int k = t >> 3, ic = (t & 7) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gi = m0 + ic + e, gk = k0 + k;
                As[ic + e][k] = (gi < M && gk < K) ? A[static_cast<int64_t>(gk) * lda + gi] : 0;
            }
        }
        // B tile: 32 x 64 elements, 8 per thread
        if (!TB) {
            const int k = t >> 3, jc = (t & 7) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gj = n0 + jc + e, gk = k0 + k;
                Bs[jc + e][k] = (gj < N && gk < K) ? B[static_cast<int64_t>(gk) * ldb + gj] : 0;
            }
        } else {
            const int j = t >> 2, kc = (t & 3) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gj = n0 + j, gk = k0 + kc + e;
                Bs[j][kc + e] = (gj < N && gk < K) ? B[static_cast<int64_t>(gj) * ldb + gk] : 0;
            }
        }
        __syncthreads();
        // A fragment: row (lane % 16), k = 8 (lane / 16) + e; B fragment:
        // column (lane % 16), same k.  Both use one k order, so the sum over
        // k is complete whatever order the hardware assigns within a step.
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            af[a] = *reinterpret_cast<const bf16x8*>(&As[32 * wr + 16 * a + (lane & 15)][8 * (lane >> 4)]);
            bfr[a] = *reinterpret_cast<const bf16x8*>(&Bs[32 * wc + 16 * a + (lane & 15)][8 * (lane >> 4)]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    // accumulator element v of a 16 x 16 tile: row 4 (lane / 16) + v, column lane % 16
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = m0 + 32 * wr + 16 * a + 4 * (lane >> 4) + v;
                const int j = n0 + 32 * wc + 16 * b + (lane & 15);
                if (i >= M || j >= N) continue;
                const int64_t o = static_cast<int64_t>(i) * ldc + j;
                const float x = acc[a][b][v];
                if constexpr (EPI == EPI_STORE) {
                    c32[o] = x;
                } else if constexpr (EPI == EPI_BIAS_GELU) {
                    const float y = x + bias[j];
                    c32[o] = y;
                    c16[o] = to_bf16(gelu(y));
                } else if constexpr (EPI == EPI_BIAS) {
                    c32[o] = x + bias[j];
                } else {
                    const float d = x * gelu_grad(aux[o]);
                    c32[o] = d;
                    c16[o] = to_bf16(d);
                }
            }
        }
    }
}

// x [B][n_in] FP32 -> xb [B][K1p] BF16 (zero padded)
__global__ void __launch_bounds__(256)
pack_input_kernel(const float* __restrict__ x, int B, int n_in, int K1p, unsigned short* __restrict__ xb) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(B) * K1p) return;
    const int b = static_cast<int>(i / K1p), k = static_cast<int>(i % K1p);
    xb[i] = k < n_in ? to_bf16(x[static_cast<int64_t>(b) * n_in + k]) : 0;
}

// One workgroup per sample: softmax over the n_out logits, softplus error
// head, per-sample loss and the output-layer gradient
//   dz_k = (q_k - p_k) / B,   ds = 2 lam (e - t) sigmoid(s) / B
// written as FP32 and BF16 rows of width N4p (padding columns zero).  With
// `t` NULL the error target is the sample's own L1 error sum_k |q_k - p_k|.
constexpr int kLossThreads = 256;
__global__ void __launch_bounds__(kLossThreads)
loss_kernel(const float* __restrict__ z, int n_out, int N4p, const float* __restrict__ p,
            const float* __restrict__ t_in, float lam, float invB, int grad,
            float* __restrict__ q_out, float* __restrict__ e_out, float* __restrict__ loss_row,
            float* __restrict__ t_used, float* __restrict__ dz32, unsigned short* __restrict__ dz16) {
    __shared__ float red[kLossThreads / 64];
    __shared__ float bc;
    const int b = blockIdx.x;
    const float* zr = z + static_cast<int64_t>(b) * N4p;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto block_reduce = [&](float v, bool is_max) -> float {
        for (int o = 32; o > 0; o >>= 1) {
            const float w = __shfl_xor(v, o);
            v = is_max ? fmaxf(v, w) : v + w;
        }
        __syncthreads();
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (tid == 0) {
            float r = red[0];
            for (int w = 1; w < kLossThreads / 64; ++w) r = is_max ? fmaxf(r, red[w]) : r + red[w];
            bc = r;
        }
        __syncthreads();
        return bc;
    };
    float mx = -INFINITY;
    for (int k = tid; k < n_out; k += kLossThreads) mx = fmaxf(mx, zr[k]);
    mx = block_reduce(mx, true);
    float se = 0.f;
    for (int k = tid; k < n_out; k += kLossThreads) se += expf(zr[k] - mx);
    se = block_reduce(se, false);
    const float lse = mx + logf(se);
    const float s = zr[n_out];
    const float e = s > 20.f ? s : log1pf(expf(s));
    float ce = 0.f, l1 = 0.f;
    const float* pr = p ? p + static_cast<int64_t>(b) * n_out : nullptr;
    for (int k = tid; k < n_out; k += kLossThreads) {
        const float q = expf(zr[k] - lse);
        if (q_out) q_out[static_cast<int64_t>(b) * n_out + k] = q;
        if (pr) {
            ce -= pr[k] * (zr[k] - lse);
            l1 += fabsf(q - pr[k]);
        }
    }
    if (e_out && tid == 0) e_out[b] = e;
    if (!pr) return;
    ce = block_reduce(ce, false);
    l1 = block_reduce(l1, false);
    const float tb = t_in ? t_in[b] : l1;
    if (tid == 0) {
        loss_row[b] = ce + lam * (e - tb) * (e - tb);
        t_used[b] = tb;
    }
    if (!grad) return;
    const float ds = 2.f * lam * (e - tb) / (1.f + expf(-s)) * invB;
    for (int k = tid; k < N4p; k += kLossThreads) {
        float d = 0.f;
        if (k < n_out) d = (expf(zr[k] - lse) - pr[k]) * invB;
        else if (k == n_out) d = ds;
        dz32[static_cast<int64_t>(b) * N4p + k] = d;
        dz16[static_cast<int64_t>(b) * N4p + k] = to_bf16(d);
    }
}

// out[j] = sum_i X[i*ld + j] over i < rows, in row order (bias gradients).
__global__ void __launch_bounds__(256)
colsum_kernel(const float* __restrict__ X, int rows, int cols, int ld, float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += X[static_cast<int64_t>(i) * ld + j];
    out[j] = s;
}

// loss = (1/B) sum_b loss_row[b], in sample order.
__global__ void __launch_bounds__(64) mean_kernel(const float* __restrict__ v, int n, float* __restrict__ out) {
    if (threadIdx.x != 0) return;
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += v[i];
    out[0] = s / static_cast<float>(n);
}

// Adam with bias correction on the FP32 masters; the BF16 copies follow.
__global__ void __launch_bounds__(256)
adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
            unsigned short* __restrict__ w16, int64_t n, float lr, float b1, float b2, float eps, float c1,
            float c2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    w16[i] = to_bf16(wi);
}

__global__ void __launch_bounds__(256)
to_bf16_kernel(const float* __restrict__ w, unsigned short* __restrict__ w16, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) w16[i] = to_bf16(w[i]);
}

int blocks(int64_t n, int t = 256) { return static_cast<int>((n + t - 1) / t); }

template <bool TA, bool TB, int EPI>
hipError_t gemm(const unsigned short* A, const unsigned short* B, int M, int N, int K, int lda, int ldb, int ldc,
                const float* bias, const float* aux, float* c32, unsigned short* c16, hipStream_t s) {
    dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile);
    gemm_kernel<TA, TB, EPI><<<grid, 256, 0, s>>>(A, B, M, N, K, lda, ldb, ldc, bias, aux, c32, c16);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Net {
    int n_in = 0, H = 0, n_out = 0, max_batch = 0;
    int K1p = 0, N4p = 0;
    int device = 0;
    int64_t step = 0;
    // offsets (elements) of the tensors in the flat parameter layout
    int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0, oW4 = 0, ob4 = 0, n_par = 0;
    float* w = nullptr;               // FP32 masters
    float* g = nullptr;               // gradients
    float* m = nullptr;               // Adam moments
    float* v = nullptr;
    unsigned short* w16 = nullptr;    // BF16 copies
    // activations
    unsigned short* xb = nullptr;     // [Bmax][K1p]
    float* a[3] = {nullptr, nullptr, nullptr};              // [Bmax][H] pre-activations
    unsigned short* h[3] = {nullptr, nullptr, nullptr};     // [Bmax][H] BF16 activations
    float* z = nullptr;               // [Bmax][N4p] logits + error head
    float* q = nullptr;               // [Bmax][n_out]
    float* e = nullptr;               // [Bmax]
    float* dz32 = nullptr;            // [Bmax][N4p]
    unsigned short* dz16 = nullptr;
    float* d32[2] = {nullptr, nullptr};                     // [Bmax][H] layer gradients
    unsigned short* d16[2] = {nullptr, nullptr};
    float* loss_row = nullptr;        // [Bmax]
    float* t_used = nullptr;          // [Bmax]
    float* loss = nullptr;            // [1]
    std::vector<void*> allocs;
};

}  // namespace mlp
}  // namespace kpm

struct kpm_mlp {
    kpm::mlp::Net net;
};

namespace kpm {
namespace mlp {
namespace {

kpm_status fail(kpm_status st, const std::string& msg) {
    set_error(msg);
    return st;
}
kpm_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? KPM_ENOMEM : KPM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define MLP_HIP(call, what)                             \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

template <typename T>
kpm_status alloc(Net& n, T** p, int64_t count) {
    void* q = nullptr;
    MLP_HIP(hipMalloc(&q, static_cast<size_t>(count) * sizeof(T)), "hipMalloc(mlp)");
    MLP_HIP(hipMemset(q, 0, static_cast<size_t>(count) * sizeof(T)), "hipMemset(mlp)");
    n.allocs.push_back(q);
    *p = static_cast<T*>(q);
    return KPM_OK;
}

void free_all(Net& n) {
    for (void* p : n.allocs) (void)hipFree(p);
    n.allocs.clear();
}

int64_t oracle_count(const Net& n) {
    return static_cast<int64_t>(n.n_in) * n.H + n.H + 2 * (static_cast<int64_t>(n.H) * n.H + n.H) +
           static_cast<int64_t>(n.H) * n.n_out + n.n_out + n.H + 1;
}

// Oracle layout (W1 [n_in x H], b1, W2, b2, W3, b3, W4 [H x n_out], b4,
// w5 [H], b5) <-> internal padded layout.  `to_internal` fills `in` (sized
// n_par, zero padding) from `orc`; otherwise the reverse.
void convert(const Net& n, const float* src, float* dst, bool to_internal) {
    const int64_t H = n.H;
    int64_t o = 0;
    auto copy = [&](int64_t ioff, int64_t count) {
        if (to_internal) std::memcpy(dst + ioff, src + o, count * sizeof(float));
        else std::memcpy(dst + o, src + ioff, count * sizeof(float));
        o += count;
    };
    copy(n.oW1, n.n_in * H);                 // W1 rows 0..n_in-1 are contiguous in W1p
    copy(n.ob1, H);
    copy(n.oW2, H * H);
    copy(n.ob2, H);
    copy(n.oW3, H * H);
    copy(n.ob3, H);
    for (int64_t r = 0; r < H; ++r) copy(n.oW4 + r * n.N4p, n.n_out);   // W4 rows
    copy(n.ob4, n.n_out);
    // w5 is column n_out of W4ext, b5 entry n_out of b4ext
    for (int64_t r = 0; r < H; ++r) {
        const int64_t io = n.oW4 + r * n.N4p + n.n_out;
        if (to_internal) dst[io] = src[o];
        else dst[o] = src[io];
        ++o;
    }
    if (to_internal) dst[n.ob4 + n.n_out] = src[o];
    else dst[o] = src[n.ob4 + n.n_out];
}

kpm_status check_dev(const Net& n) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(KPM_EDEVICE, "hipGetDevice failed");
    if (dev != n.device) return fail(KPM_EINVAL, "current device differs from the network's device");
    return KPM_OK;
}

kpm_status forward(Net& n, const float* x, int B, hipStream_t s) {
    const unsigned short* W1 = n.w16 + n.oW1;
    const unsigned short* W2 = n.w16 + n.oW2;
    const unsigned short* W3 = n.w16 + n.oW3;
    const unsigned short* W4 = n.w16 + n.oW4;
    const int H = n.H;
    pack_input_kernel<<<blocks(static_cast<int64_t>(B) * n.K1p), 256, 0, s>>>(x, B, n.n_in, n.K1p, n.xb);
    MLP_HIP(hipGetLastError(), "pack kernel");
    MLP_HIP((gemm<false, false, EPI_BIAS_GELU>(n.xb, W1, B, H, n.K1p, n.K1p, H, H, n.w + n.ob1, nullptr, n.a[0],
                                               n.h[0], s)), "gemm layer 1");
    MLP_HIP((gemm<false, false, EPI_BIAS_GELU>(n.h[0], W2, B, H, H, H, H, H, n.w + n.ob2, nullptr, n.a[1], n.h[1],
                                               s)), "gemm layer 2");
    MLP_HIP((gemm<false, false, EPI_BIAS_GELU>(n.h[1], W3, B, H, H, H, H, H, n.w + n.ob3, nullptr, n.a[2], n.h[2],
                                               s)), "gemm layer 3");
    MLP_HIP((gemm<false, false, EPI_BIAS>(n.h[2], W4, B, n.N4p, H, H, n.N4p, n.N4p, n.w + n.ob4, nullptr, n.z,
                                          nullptr, s)), "gemm output");
    return KPM_OK;
}

// Gradients of the loss for the batch in n.z / activations into n.g.
kpm_status backward(Net& n, int B, hipStream_t s) {
    const int H = n.H;
    float* g = n.g;
    // output layer (W4ext, b4ext)
    MLP_HIP((gemm<true, false, EPI_STORE>(n.h[2], n.dz16, H, n.N4p, B, H, n.N4p, n.N4p, nullptr, nullptr,
                                          g + n.oW4, nullptr, s)), "gemm dW4");
    colsum_kernel<<<blocks(n.N4p), 256, 0, s>>>(n.dz32, B, n.N4p, n.N4p, g + n.ob4);
    MLP_HIP(hipGetLastError(), "colsum");
    // dh3 = dz W4ext^T, da3 = dh3 * gelu'(a3)
    MLP_HIP((gemm<false, true, EPI_DGELU>(n.dz16, n.w16 + n.oW4, B, H, n.N4p, n.N4p, n.N4p, H, nullptr, n.a[2],
                                          n.d32[0], n.d16[0], s)), "gemm dh3");
    const int64_t oW[3] = {n.oW1, n.oW2, n.oW3};
    const int64_t ob[3] = {n.ob1, n.ob2, n.ob3};
    int cur = 0;
    for (int l = 2; l >= 0; --l) {
        // dW_l = h_{l-1}^T da_l (h_{-1} = x), db_l = colsum(da_l)
        const unsigned short* hin = l > 0 ? n.h[l - 1] : n.xb;
        const int kin = l > 0 ? H : n.K1p;
        MLP_HIP((gemm<true, false, EPI_STORE>(hin, n.d16[cur], kin, H, B, kin, H, H, nullptr, nullptr, g + oW[l],
                                              nullptr, s)), "gemm dW");
        colsum_kernel<<<blocks(H), 256, 0, s>>>(n.d32[cur], B, H, H, g + ob[l]);
        MLP_HIP(hipGetLastError(), "colsum");
        if (l > 0) {
            // da_{l-1} = (da_l W_l^T) * gelu'(a_{l-1})
            MLP_HIP((gemm<false, true, EPI_DGELU>(n.d16[cur], n.w16 + oW[l], B, H, H, H, H, H, nullptr, n.a[l - 1],
                                                  n.d32[cur ^ 1], n.d16[cur ^ 1], s)), "gemm dh");
            cur ^= 1;
        }
    }
    return KPM_OK;
}

}  // namespace
}  // namespace mlp
}  // namespace kpm

using namespace kpm::mlp;

extern "C" {

kpm_status kpm_mlp_create(int32_t n_in, int32_t hidden, int32_t n_out, int32_t max_batch, kpm_mlp** out) {
    kpm::set_error("");
    if (!out) return fail(KPM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_in <= 0 || hidden <= 0 || n_out <= 0 || max_batch <= 0)
        return fail(KPM_EINVAL, "sizes must be positive");
    if (n_in > 65536 || hidden > 65536 || n_out > 65536 || max_batch > (1 << 22))
        return fail(KPM_EINVAL, "sizes too large");
    auto* net = new kpm_mlp();
    Net& n = net->net;
    n.n_in = n_in;
    n.H = hidden;
    n.n_out = n_out;
    n.max_batch = max_batch;
    n.K1p = (n_in + 31) / 32 * 32;
    n.N4p = (n_out + 1 + 15) / 16 * 16;
    if (hipGetDevice(&n.device) != hipSuccess) {
        delete net;
        return fail(KPM_EDEVICE, "hipGetDevice failed");
    }
    const int64_t H = hidden;
    n.oW1 = 0;
    n.ob1 = n.oW1 + static_cast<int64_t>(n.K1p) * H;
    n.oW2 = n.ob1 + H;
    n.ob2 = n.oW2 + H * H;
    n.oW3 = n.ob2 + H;
    n.ob3 = n.oW3 + H * H;
    n.oW4 = n.ob3 + H;
    n.ob4 = n.oW4 + H * n.N4p;
    n.n_par = n.ob4 + n.N4p;
    const int64_t Bm = max_batch;
    kpm_status st = KPM_OK;
    if ((st = alloc(n, &n.w, n.n_par)) != KPM_OK || (st = alloc(n, &n.g, n.n_par)) != KPM_OK ||
        (st = alloc(n, &n.m, n.n_par)) != KPM_OK || (st = alloc(n, &n.v, n.n_par)) != KPM_OK ||
        (st = alloc(n, &n.w16, n.n_par)) != KPM_OK || (st = alloc(n, &n.xb, Bm * n.K1p)) != KPM_OK ||
        (st = alloc(n, &n.z, Bm * n.N4p)) != KPM_OK || (st = alloc(n, &n.q, Bm * n_out)) != KPM_OK ||
        (st = alloc(n, &n.e, Bm)) != KPM_OK || (st = alloc(n, &n.dz32, Bm * n.N4p)) != KPM_OK ||
        (st = alloc(n, &n.dz16, Bm * n.N4p)) != KPM_OK || (st = alloc(n, &n.loss_row, Bm)) != KPM_OK ||
        (st = alloc(n, &n.t_used, Bm)) != KPM_OK || (st = alloc(n, &n.loss, 1)) != KPM_OK) {
        free_all(n);
        delete net;
        return st;
    }
    for (int l = 0; l < 3 && st == KPM_OK; ++l) {
        if ((st = alloc(n, &n.a[l], Bm * H)) == KPM_OK) st = alloc(n, &n.h[l], Bm * H);
    }
    for (int l = 0; l < 2 && st == KPM_OK; ++l) {
        if ((st = alloc(n, &n.d32[l], Bm * H)) == KPM_OK) st = alloc(n, &n.d16[l], Bm * H);
    }
    if (st != KPM_OK) {
        free_all(n);
        delete net;
        return st;
    }
    *out = net;
    return KPM_OK;
}

void kpm_mlp_destroy(kpm_mlp* net) {
    if (!net) return;
    (void)hipDeviceSynchronize();
    free_all(net->net);
    delete net;
}

kpm_status kpm_mlp_param_count(const kpm_mlp* net, int64_t* count) {
    kpm::set_error("");
    if (!net || !count) return fail(KPM_EINVAL, "net or count is NULL");
    *count = oracle_count(net->net);
    return KPM_OK;
}

kpm_status kpm_mlp_set_params(kpm_mlp* net, const float* params) {
    kpm::set_error("");
    if (!net || !params) return fail(KPM_EINVAL, "net or params is NULL");
    Net& n = net->net;
    kpm_status st = check_dev(n);
    if (st != KPM_OK) return st;
    for (int64_t i = 0; i < oracle_count(n); ++i)
        if (!std::isfinite(params[i])) return fail(KPM_EINVAL, "parameters must be finite");
    std::vector<float> in(n.n_par, 0.0f);
    convert(n, params, in.data(), true);
    MLP_HIP(hipDeviceSynchronize(), "synchronise");
    MLP_HIP(hipMemcpy(n.w, in.data(), n.n_par * sizeof(float), hipMemcpyHostToDevice), "copy params");
    MLP_HIP(hipMemset(n.m, 0, n.n_par * sizeof(float)), "reset Adam");
    MLP_HIP(hipMemset(n.v, 0, n.n_par * sizeof(float)), "reset Adam");
    MLP_HIP(hipMemset(n.g, 0, n.n_par * sizeof(float)), "reset grads");
    to_bf16_kernel<<<blocks(n.n_par), 256>>>(n.w, n.w16, n.n_par);
    MLP_HIP(hipGetLastError(), "bf16 kernel");
    MLP_HIP(hipDeviceSynchronize(), "synchronise");
    n.step = 0;
    return KPM_OK;
}

static kpm_status export_flat(const Net& n, const float* dev, float* host) {
    std::vector<float> in(n.n_par);
    MLP_HIP(hipDeviceSynchronize(), "synchronise");
    MLP_HIP(hipMemcpy(in.data(), dev, n.n_par * sizeof(float), hipMemcpyDeviceToHost), "copy params");
    convert(n, in.data(), host, false);
    return KPM_OK;
}

kpm_status kpm_mlp_get_params(const kpm_mlp* net, float* params) {
    kpm::set_error("");
    if (!net || !params) return fail(KPM_EINVAL, "net or params is NULL");
    kpm_status st = check_dev(net->net);
    if (st != KPM_OK) return st;
    return export_flat(net->net, net->net.w, params);
}

kpm_status kpm_mlp_get_grads(const kpm_mlp* net, float* grads) {
    kpm::set_error("");
    if (!net || !grads) return fail(KPM_EINVAL, "net or grads is NULL");
    kpm_status st = check_dev(net->net);
    if (st != KPM_OK) return st;
    return export_flat(net->net, net->net.g, grads);
}

kpm_status kpm_mlp_forward(kpm_mlp* net, const float* x, int32_t B, float* q, float* e, void* stream) {
    kpm::set_error("");
    if (!net || !x) return fail(KPM_EINVAL, "net or x is NULL");
    Net& n = net->net;
    if (B <= 0 || B > n.max_batch) return fail(KPM_EINVAL, "batch size out of range");
    kpm_status st = check_dev(n);
    if (st != KPM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = forward(n, x, B, s)) != KPM_OK) return st;
    loss_kernel<<<B, kLossThreads, 0, s>>>(n.z, n.n_out, n.N4p, nullptr, nullptr, 0.f, 1.f / B, 0, q ? q : n.q,
                                           e ? e : n.e, nullptr, nullptr, nullptr, nullptr);
    MLP_HIP(hipGetLastError(), "softmax kernel");
    return KPM_OK;
}

kpm_status kpm_mlp_backward(kpm_mlp* net, const float* x, const float* p, const float* t, int32_t B, float lam,
                            float* loss, void* stream) {
    kpm::set_error("");
    if (!net || !x || !p) return fail(KPM_EINVAL, "net, x or p is NULL");
    Net& n = net->net;
    if (B <= 0 || B > n.max_batch) return fail(KPM_EINVAL, "batch size out of range");
    if (!(lam >= 0.0f) || !std::isfinite(lam)) return fail(KPM_EINVAL, "lam must be finite and >= 0");
    kpm_status st = check_dev(n);
    if (st != KPM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = forward(n, x, B, s)) != KPM_OK) return st;
    loss_kernel<<<B, kLossThreads, 0, s>>>(n.z, n.n_out, n.N4p, p, t, lam, 1.f / B, 1, n.q, n.e, n.loss_row,
                                           n.t_used, n.dz32, n.dz16);
    MLP_HIP(hipGetLastError(), "loss kernel");
    mean_kernel<<<1, 64, 0, s>>>(n.loss_row, B, loss ? loss : n.loss);
    MLP_HIP(hipGetLastError(), "mean kernel");
    return backward(n, B, s);
}

kpm_status kpm_mlp_adam_step(kpm_mlp* net, float lr, float beta1, float beta2, float eps, void* stream) {
    kpm::set_error("");
    if (!net) return fail(KPM_EINVAL, "net is NULL");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(KPM_EINVAL, "need lr > 0, 0 <= beta < 1, eps > 0");
    Net& n = net->net;
    kpm_status st = check_dev(n);
    if (st != KPM_OK) return st;
    ++n.step;
    const float c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), static_cast<double>(n.step)));
    const float c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), static_cast<double>(n.step)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    adam_kernel<<<blocks(n.n_par), 256, 0, s>>>(n.w, n.g, n.m, n.v, n.w16, n.n_par, lr, beta1, beta2, eps, c1, c2);
    MLP_HIP(hipGetLastError(), "adam kernel");
    return KPM_OK;
}

kpm_status kpm_mlp_train_step(kpm_mlp* net, const float* x, const float* p, const float* t, int32_t B, float lam,
                              float lr, float* loss, void* stream) {
    kpm_status st = kpm_mlp_backward(net, x, p, t, B, lam, loss, stream);
    if (st != KPM_OK) return st;
    return kpm_mlp_adam_step(net, lr, 0.9f, 0.999f, 1e-8f, stream);
}

kpm_status kpm_mlp_gemm_bf16(const uint16_t* A, const uint16_t* B, int32_t M, int32_t N, int32_t K, int32_t trans_a,
                             int32_t trans_b, float* C, void* stream) {
    kpm::set_error("");
    if (!A || !B || !C) return fail(KPM_EINVAL, "A, B or C is NULL");
    if (M <= 0 || N <= 0 || K <= 0) return fail(KPM_EINVAL, "sizes must be positive");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int lda = trans_a ? M : K, ldb = trans_b ? K : N;
    hipError_t e;
    if (!trans_a && !trans_b) e = gemm<false, false, EPI_STORE>(A, B, M, N, K, lda, ldb, N, nullptr, nullptr, C, nullptr, s);
    else if (trans_a && !trans_b) e = gemm<true, false, EPI_STORE>(A, B, M, N, K, lda, ldb, N, nullptr, nullptr, C, nullptr, s);
    else if (!trans_a && trans_b) e = gemm<false, true, EPI_STORE>(A, B, M, N, K, lda, ldb, N, nullptr, nullptr, C, nullptr, s);
    else return fail(KPM_ENOTSUP, "both operands transposed is not supported");
    MLP_HIP(e, "gemm kernel");
    return KPM_OK;
}

}  // extern "C"
