// crk_learned.hip -- learned troubled-cell indicator for the blending limiter:
// a multilayer perceptron nin -> H -> H -> 1 (ReLU, output alpha_max *
// sigmoid) on the modal energy fractions of rho*p, with BF16 parameters and
// FP32 arithmetic; its training kernels (loss gradient, Adam), the training
// labels (a-posteriori troubled elements) and the inference that replaces the
// modal blending coefficient, falling back to it where the network is not
// trusted.  Parameter vector layout (P values):
//   W1[H][nin], b1[H], W2[H][H], b2[H], W3[H], b3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/crk.h"
#include "crk_kernels.hpp"

using namespace crk;

namespace crk {
const char *set_error(crk_status st, const char *msg);
}

namespace {

constexpr int NIN = 16;   // (N+1)^2 features of a degree-3 quadrilateral
constexpr int HID = 64;
constexpr long NPAR = (long)HID * NIN + HID + (long)HID * HID + HID + HID + 1;
constexpr int SB = 32;    // samples per workgroup of the gradient kernel

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct MlpView {
    const uint16_t *W1, *b1, *W2, *b2, *W3, *b3;
};
__device__ __forceinline__ MlpView mlp_view(const uint16_t *th)
{
    MlpView v;
    v.W1 = th;
    v.b1 = v.W1 + HID * NIN;
    v.W2 = v.b1 + HID;
    v.b2 = v.W2 + HID * HID;
    v.W3 = v.b2 + HID;
    v.b3 = v.W3 + HID;
    return v;
}

// z of one sample; the weights are read at lane-uniform addresses (scalar loads)
__device__ __forceinline__ float mlp_z(const MlpView &w, const float *x)
{
    float h1[HID];
#pragma unroll
    for (int j = 0; j < HID; ++j) {
        float a = bf2f(w.b1[j]);
#pragma unroll
        for (int c = 0; c < NIN; ++c) a = fmaf(bf2f(w.W1[j * NIN + c]), x[c], a);
        h1[j] = a > 0.f ? a : 0.f;
    }
    float z = bf2f(w.b3[0]);
    for (int k = 0; k < HID; ++k) {
        float a = bf2f(w.b2[k]);
#pragma unroll
        for (int j = 0; j < HID; ++j) a = fmaf(bf2f(w.W2[k * HID + j]), h1[j], a);
        z = fmaf(bf2f(w.W3[k]), a > 0.f ? a : 0.f, z);
    }
    return z;
}

__global__ void __launch_bounds__(256) k_mlp_forward(const uint16_t *theta, const float *x, long n, float alpha_max,
                                                     float *z_out, double *alpha_out)
{
    const long s = (long)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const MlpView w = mlp_view(theta);
    float xs[NIN];
#pragma unroll
    for (int c = 0; c < NIN; ++c) xs[c] = x[s * NIN + c];
    const float z = mlp_z(w, xs);
    if (z_out) z_out[s] = z;
    if (alpha_out) alpha_out[s] = (double)alpha_max / (1.0 + exp(-(double)z));
}

// Gradient of the mean binary cross-entropy of sigmoid(z) against y over
// n_total samples: one workgroup per SB samples writes its partial gradient.
__global__ void __launch_bounds__(256) k_mlp_grad(const uint16_t *theta, const float *x, const float *y, long n,
                                                  long n_total, float *partial, float *partial_loss)
{
    __shared__ float xs[SB][NIN];
    __shared__ float A1[SB][HID], A2[SB][HID], D1[SB][HID], D2[SB][HID];
    __shared__ float dz[SB], ls[SB];
    const int tid = threadIdx.x;
    const long s0 = (long)blockIdx.x * SB;
    const MlpView w = mlp_view(theta);
    for (int i = tid; i < SB * NIN; i += 256) {
        const int s = i / NIN, c = i - s * NIN;
        xs[s][c] = (s0 + s < n) ? x[(s0 + s) * NIN + c] : 0.f;
    }
    __syncthreads();
    for (int i = tid; i < SB * HID; i += 256) {
        const int s = i / HID, j = i - s * HID;
        float a = bf2f(w.b1[j]);
#pragma unroll
        for (int c = 0; c < NIN; ++c) a = fmaf(bf2f(w.W1[j * NIN + c]), xs[s][c], a);
        A1[s][j] = a;
    }
    __syncthreads();
    for (int i = tid; i < SB * HID; i += 256) {
        const int s = i / HID, k = i - s * HID;
        float a = bf2f(w.b2[k]);
        for (int j = 0; j < HID; ++j) a = fmaf(bf2f(w.W2[k * HID + j]), fmaxf(A1[s][j], 0.f), a);
        A2[s][k] = a;
    }
    __syncthreads();
    if (tid < SB) {
        const int s = tid;
        float z = bf2f(w.b3[0]);
        for (int k = 0; k < HID; ++k) z = fmaf(bf2f(w.W3[k]), fmaxf(A2[s][k], 0.f), z);
        const bool in = s0 + s < n;
        const float yy = in ? y[s0 + s] : 0.f;
        const float sg = 1.f / (1.f + expf(-z));
        dz[s] = in ? (sg - yy) / (float)n_total : 0.f;
        // BCE with logits, stable form: log(1 + e^z) - y z
        ls[s] = in ? ((z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z))) - yy * z) : 0.f;
    }
    __syncthreads();
    for (int i = tid; i < SB * HID; i += 256) {
        const int s = i / HID, k = i - s * HID;
        D2[s][k] = A2[s][k] > 0.f ? dz[s] * bf2f(w.W3[k]) : 0.f;
    }
    __syncthreads();
    for (int i = tid; i < SB * HID; i += 256) {
        const int s = i / HID, j = i - s * HID;
        float a = 0.f;
        for (int k = 0; k < HID; ++k) a = fmaf(bf2f(w.W2[k * HID + j]), D2[s][k], a);
        D1[s][j] = A1[s][j] > 0.f ? a : 0.f;
    }
    __syncthreads();
    float *g = partial + (long)blockIdx.x * NPAR;
    float *gW1 = g, *gb1 = gW1 + HID * NIN, *gW2 = gb1 + HID, *gb2 = gW2 + HID * HID, *gW3 = gb2 + HID, *gb3 = gW3 + HID;
    for (int i = tid; i < HID * NIN; i += 256) {
        const int j = i / NIN, c = i - j * NIN;
        float a = 0.f;
        for (int s = 0; s < SB; ++s) a = fmaf(D1[s][j], xs[s][c], a);
        gW1[i] = a;
    }
    for (int i = tid; i < HID * HID; i += 256) {
        const int k = i / HID, j = i - k * HID;
        float a = 0.f;
        for (int s = 0; s < SB; ++s) a = fmaf(D2[s][k], fmaxf(A1[s][j], 0.f), a);
        gW2[i] = a;
    }
    if (tid < HID) {
        float a1 = 0.f, a2 = 0.f, a3 = 0.f;
        for (int s = 0; s < SB; ++s) {
            a1 += D1[s][tid];
            a2 += D2[s][tid];
            a3 = fmaf(dz[s], fmaxf(A2[s][tid], 0.f), a3);
        }
        gb1[tid] = a1;
        gb2[tid] = a2;
        gW3[tid] = a3;
    }
    if (tid == 0) {
        float a = 0.f, l = 0.f;
        for (int s = 0; s < SB; ++s) {
            a += dz[s];
            l += ls[s];
        }
        gb3[0] = a;
        partial_loss[blockIdx.x] = l;
    }
}

// sum of the partials in workgroup order (deterministic)
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *partial, const float *partial_loss, int nblocks,
                                                    long n_total, float *grad, float *loss)
{
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p < NPAR) {
        float a = 0.f;
        for (int b = 0; b < nblocks; ++b) a += partial[(long)b * NPAR + p];
        grad[p] = a;
    } else if (p == NPAR && loss) {
        float l = 0.f;
        for (int b = 0; b < nblocks; ++b) l += partial_loss[b];
        *loss = l / (float)n_total;
    }
}

__global__ void __launch_bounds__(256) k_adam(long count, float *theta, float *m, float *v, const float *g, float lr,
                                              float b1, float b2, float eps, float c1, float c2, uint16_t *theta_bf16)
{
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float th = theta[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    theta[k] = th;
    if (theta_bf16) theta_bf16[k] = f2bf(th);
}

__global__ void __launch_bounds__(256) k_to_bf16(long count, const float *x, uint16_t *y)
{
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k < count) y[k] = f2bf(x[k]);
}

// Blending coefficient from the network where it is trusted: features inside
// the training range [lo, hi] and a finite output; elsewhere the modal
// coefficient already in alpha_raw stays.  alpha < alpha_min is cut to 0 as
// for the modal indicator.
// Inference for the blending coefficient on the matrix cores.  One
// wavefront takes tiles of 16 elements and forms each layer transposed,
// Y^T = W X^T: the BF16 weights are the exact A operand, and every FP32
// activation enters the B operand as the sum of three BF16 parts
// (x = hi + mid + lo to within 2^-24 |x|), so each product is exact in FP32
// and the result is the FP32 network up to the summation order.  The first
// layer (16 inputs) uses v_mfma_f32_16x16x16_bf16, operand layout (lane l,
// i = 0..3): A[l % 16][4 (l / 16) + i], B[4 (l / 16) + i][l % 16],
// D[4 (l / 16) + i][l % 16]; a layer's D is therefore already a B operand of
// the next layer.  The second layer (64 hidden inputs) uses the K = 32 form
// v_mfma_f32_16x16x32_bf16 on two 16-row D blocks at a time: a lane's eight
// B values are its four rows of each block, and its eight A values are the
// weights of the same hidden units (whatever hidden unit an operand slot
// carries, A and B carry the same one, so the sum runs over the block pair).
// The weights stay in registers while the wavefront walks its tiles.
typedef short mx_s4 __attribute__((ext_vector_type(4)));
typedef float mx_f4 __attribute__((ext_vector_type(4)));

// x = hi + mid + lo in BF16 (round to nearest even: the hardware conversion)
__device__ __forceinline__ void split3(const float *x, mx_s4 &h, mx_s4 &m, mx_s4 &l)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const __bf16 bh = (__bf16)x[i];
        const float r1 = x[i] - (float)bh;
        const __bf16 bm = (__bf16)r1;
        const float r2 = r1 - (float)bm;
        h[i] = __builtin_bit_cast(short, bh);
        m[i] = __builtin_bit_cast(short, bm);
        l[i] = __builtin_bit_cast(short, (__bf16)r2);
    }
}

__device__ __forceinline__ mx_f4 mfma3(const mx_s4 &a, const mx_s4 &bh, const mx_s4 &bm, const mx_s4 &bl, mx_f4 acc)
{
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bm, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bh, acc, 0, 0, 0);
}

typedef __bf16 mx_b8 __attribute__((ext_vector_type(8)));
typedef short mx_s8 __attribute__((ext_vector_type(8)));

// two 4-value operands of the K = 16 form as one 8-value operand of the
// K = 32 form, reinterpreted as a whole vector (built element by element
// from bit-cast BF16 values, the operand reached the instruction wrongly
// packed with this compiler, although its bits read back unchanged)
__device__ __forceinline__ mx_b8 join8(const mx_s4 &p, const mx_s4 &q)
{
    const mx_s8 t = __builtin_shufflevector(p, q, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(mx_b8, t);
}

__device__ __forceinline__ mx_f4 mfma3k32(const mx_b8 &a, const mx_b8 &bh, const mx_b8 &bm, const mx_b8 &bl, mx_f4 acc)
{
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bm, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc, 0, 0, 0);
}

constexpr int MX_TILE = 16;
static_assert(NIN == 16 && HID == 64, "the tiling below is written for 16 inputs and 64 hidden units");

__global__ void __launch_bounds__(256) k_mlp_alpha(const uint16_t *theta, const float *features, const float *lo,
                                                   const float *hi, long nelem, double alpha_max, double alpha_min,
                                                   double *alpha_raw, const crk::Tables t, int epb, int *tiles)
{
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kq = lane >> 4;
    const long wave = ((long)blockIdx.x * 256 + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * 256) >> 6;
    const long ntiles = (nelem + MX_TILE - 1) / MX_TILE;
    if (wave >= ntiles) return;                       // uniform per wavefront
    const MlpView w = mlp_view(theta);
    // per-lane weights: A blocks of W1 (hidden 16b + col, inputs 4kq..) and
    // W2 (out 16c + col, in 16b + 4kq ..), biases and W3 of the hidden units
    // 16b + 4kq + i this lane holds in D
    mx_s4 A1[4], A2[4][4];
    float B1[4][4], B2[4][4], W3[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            A1[b][i] = (short)w.W1[(16 * b + col) * NIN + 4 * kq + i];
            B1[b][i] = bf2f(w.b1[16 * b + 4 * kq + i]);
            B2[b][i] = bf2f(w.b2[16 * b + 4 * kq + i]);
            W3[b][i] = bf2f(w.W3[16 * b + 4 * kq + i]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i) A2[c][b][i] = (short)w.W2[(16 * c + col) * HID + 16 * b + 4 * kq + i];
    }
    mx_b8 A2k[4][2];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) A2k[c][kb] = join8(A2[c][2 * kb], A2[c][2 * kb + 1]);
    const float b3 = bf2f(w.b3[0]);
    float flo[4], fhi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { flo[i] = lo[4 * kq + i]; fhi[i] = hi[4 * kq + i]; }

    for (long tile = wave; tile < ntiles; tile += nwaves) {
        const long e = tile * MX_TILE + col;
        const bool ev = e < nelem;
        float x[4];
        bool inside = true;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            x[i] = ev ? features[e * NIN + 4 * kq + i] : 0.f;
            inside &= (x[i] >= flo[i]) && (x[i] <= fhi[i]);
        }
        // the four lanes of an element (col, col + 16, col + 32, col + 48)
        inside = inside && __shfl_xor((int)inside, 16) && __shfl_xor((int)inside, 32);
        mx_s4 xh, xm, xl;
        split3(x, xh, xm, xl);
        // layer 1: H1^T block b = W1[16b.., :] X^T
        float h1[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            mx_f4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma3(A1[b], xh, xm, xl, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[i] + B1[b][i];
                h1[b][i] = v > 0.f ? v : 0.f;
            }
        }
        mx_s4 hh[4], hm[4], hl[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) split3(h1[b], hh[b], hm[b], hl[b]);
        // layer 2 (K = 32: hidden blocks 2 kb and 2 kb + 1 together) and the
        // output layer's partial dot product
        mx_b8 kh[2], km[2], kl[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            kh[kb] = join8(hh[2 * kb], hh[2 * kb + 1]);
            km[kb] = join8(hm[2 * kb], hm[2 * kb + 1]);
            kl[kb] = join8(hl[2 * kb], hl[2 * kb + 1]);
        }
        float z = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            mx_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) acc = mfma3k32(A2k[c][kb], kh[kb], km[kb], kl[kb], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[i] + B2[c][i];
                z = fmaf(W3[c][i], v > 0.f ? v : 0.f, z);
            }
        }
        z += __shfl_xor(z, 16);
        z += __shfl_xor(z, 32);
        z += b3;
        if (kq == 0 && ev && inside && isfinite(z)) {
            double a = alpha_max / (1.0 + exp(-(double)z));
            if (a < alpha_min) a = 0.0;
            alpha_raw[e] = a;
            // local-phase tile flags of the pipelined step (2D meshes)
            if (tiles != nullptr && a > 0.0) crk::mark_tiles<2>(t, e, epb, tiles);
        }
    }
}

// Troubled-element labels: the unlimited update uh leaves the range of rho or
// p over the element and its face neighbours in un by more than tol
// (relative), or is inadmissible.  One lane per node.
template <typename real, int N>
__global__ void __launch_bounds__(BLOCK) k_labels(const Tables t, const void *un_, const void *uh_, double tol, float *labels)
{
    constexpr int NP = (N + 1) * (N + 1);
    constexpr int EPB = BLOCK / NP;
    __shared__ double red[4][BLOCK];
    __shared__ int bad[BLOCK];
    const int tid = threadIdx.x;
    int le = tid / NP;
    const int node = tid - le * NP;
    const long e = (long)blockIdx.x * EPB + le;
    const bool valid = (le < EPB) && (e < t.nelem);
    if (le >= EPB) le = 0;
    const long es = valid ? e : 0;
    const long E = t.nelem;
    const real *un = (const real *)un_, *uh = (const real *)uh_;
    auto pres = [&](const real *u, long el) {
        const double r = u[((long)0 * E + el) * NP + node], m1 = u[((long)1 * E + el) * NP + node];
        const double m2 = u[((long)2 * E + el) * NP + node], En = u[((long)3 * E + el) * NP + node];
        return (t.gamma - 1.0) * (En - 0.5 * (m1 * m1 + m2 * m2) / r);
    };
    const Nbrs nb = neighbours<2>(t, es);
    long list[5] = {es, nb.n[0][0], nb.n[0][1], nb.n[1][0], nb.n[1][1]};
    double rmin = INFINITY, rmax = -INFINITY, pmin = INFINITY, pmax = -INFINITY;
    for (int k = 0; k < 5; ++k) {
        const double r = un[((long)0 * E + list[k]) * NP + node], p = pres(un, list[k]);
        rmin = fmin(rmin, r);
        rmax = fmax(rmax, r);
        pmin = fmin(pmin, p);
        pmax = fmax(pmax, p);
    }
    red[0][tid] = rmin; red[1][tid] = rmax; red[2][tid] = pmin; red[3][tid] = pmax;
    __syncthreads();
    const int b0 = le * NP;
    for (int q = 0; q < NP; ++q) {
        rmin = fmin(rmin, red[0][b0 + q]);
        rmax = fmax(rmax, red[1][b0 + q]);
        pmin = fmin(pmin, red[2][b0 + q]);
        pmax = fmax(pmax, red[3][b0 + q]);
    }
    int flag = 0;
    for (int v = 0; v < 4; ++v)
        if (!isfinite((double)uh[((long)v * E + es) * NP + node])) flag = 1;
    const double r = uh[((long)0 * E + es) * NP + node], p = pres(uh, es);
    if (!(r > 0.0) || !(p > 0.0)) flag = 1;
    if (r < rmin * (1.0 - tol) || r > rmax * (1.0 + tol)) flag = 1;
    if (p < pmin * (1.0 - tol) || p > pmax * (1.0 + tol)) flag = 1;
    bad[tid] = flag;
    __syncthreads();
    if (!valid || node != 0) return;
    int any = 0;
    for (int q = 0; q < NP; ++q) any |= bad[b0 + q];
    labels[e] = any ? 1.f : 0.f;
}

crk_status hip_err(hipError_t e, const char *where)
{
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    set_error(CRK_ERR_HIP, m.c_str());
    return CRK_ERR_HIP;
}

crk_status check_shape(int nin, int hidden)
{
    if (nin != NIN || hidden != HID) {
        set_error(CRK_ERR_UNSUPPORTED, "the network is compiled for 16 inputs and 64 hidden units");
        return CRK_ERR_UNSUPPORTED;
    }
    return CRK_OK;
}

inline unsigned blocks(long n, int b) { return (unsigned)((n + b - 1) / b); }

} // namespace

namespace crk {
// used by crk_api.cpp: learned blending coefficients over the modal ones
hipError_t launch_mlp_alpha(const uint16_t *theta, const float *features, const float *lo, const float *hi, long nelem,
                            double alpha_max, double alpha_min, double *alpha_raw, const Tables *t, int *flags,
                            hipStream_t s)
{
    // four wavefronts per workgroup, each walking tiles of 16 elements; at
    // most two wavefronts per SIMD of the 256 CUs (the register budget)
    const long tiles = (nelem + MX_TILE - 1) / MX_TILE;
    long g = (tiles + 3) / 4;
    if (g > 256 * 2) g = 256 * 2;
    // flags: local-phase tile flags of the 2D mesh described by *t, or nullptr
    const bool mark = flags != nullptr && t != nullptr;
    const Tables tt = mark ? *t : Tables{};
    const int epb = mark ? tile_block_rt((int)tt.nnode) / (int)tt.nnode : 1;
    hipLaunchKernelGGL(k_mlp_alpha, dim3((unsigned)g), dim3(256), 0, s, theta, features, lo, hi, nelem, alpha_max,
                       alpha_min, alpha_raw, tt, epb, mark ? flags : nullptr);
    return hipGetLastError();
}
hipError_t launch_labels(const Tables &t, int prec, const void *un, const void *uh, double tol, float *labels, hipStream_t s)
{
    const int NP = t.nnode;
    const unsigned g = blocks(t.nelem, BLOCK / NP);
    if (t.dim != 2) return hipErrorInvalidValue;
#define CRK_LAB(R, NN) hipLaunchKernelGGL((k_labels<R, NN>), dim3(g), dim3(BLOCK), 0, s, t, un, uh, tol, labels)
    if (prec == CRK_FP64) {
        switch (t.N) { case 1: CRK_LAB(double, 1); break; case 2: CRK_LAB(double, 2); break;
                       case 3: CRK_LAB(double, 3); break; default: CRK_LAB(double, 4); }
    } else {
        switch (t.N) { case 1: CRK_LAB(float, 1); break; case 2: CRK_LAB(float, 2); break;
                       case 3: CRK_LAB(float, 3); break; default: CRK_LAB(float, 4); }
    }
#undef CRK_LAB
    return hipGetLastError();
}
} // namespace crk

extern "C" {

crk_status crk_mlp_param_count(int nin, int hidden, int64_t *count)
{
    if (!count) { set_error(CRK_ERR_ARG, "null argument"); return CRK_ERR_ARG; }
    crk_status st = check_shape(nin, hidden);
    if (st) return st;
    *count = NPAR;
    return CRK_OK;
}

crk_status crk_mlp_forward(int nin, int hidden, const uint16_t *theta_bf16, const float *x, int64_t n, double alpha_max,
                           float *z, double *alpha, crk_stream stream)
{
    crk_status st = check_shape(nin, hidden);
    if (st) return st;
    if (!theta_bf16 || !x || n < 0) { set_error(CRK_ERR_ARG, "null argument"); return CRK_ERR_ARG; }
    if (n == 0) return CRK_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, theta_bf16, x, (long)n,
                       (float)alpha_max, z, alpha);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CRK_OK : hip_err(e, "crk_mlp_forward");
}

crk_status crk_mlp_grad_workspace_bytes(int nin, int hidden, int64_t n, size_t *bytes)
{
    crk_status st = check_shape(nin, hidden);
    if (st) return st;
    if (!bytes || n < 0) { set_error(CRK_ERR_ARG, "bad argument"); return CRK_ERR_ARG; }
    const long nb = (long)blocks(n, SB);
    *bytes = ((size_t)nb * NPAR * sizeof(float) + 255) / 256 * 256 + (size_t)nb * sizeof(float);
    return CRK_OK;
}

crk_status crk_mlp_loss_grad(int nin, int hidden, const uint16_t *theta_bf16, const float *x, const float *y, int64_t n,
                             float *grad, float *loss, void *workspace, size_t ws_bytes, crk_stream stream)
{
    crk_status st = check_shape(nin, hidden);
    if (st) return st;
    if (!theta_bf16 || !x || !y || !grad || !workspace || n < 1) { set_error(CRK_ERR_ARG, "null argument"); return CRK_ERR_ARG; }
    size_t need = 0;
    crk_mlp_grad_workspace_bytes(nin, hidden, n, &need);
    if (ws_bytes < need) { set_error(CRK_ERR_ARG, "workspace too small"); return CRK_ERR_ARG; }
    const unsigned nb = blocks(n, SB);
    float *part = (float *)workspace;
    float *pl = (float *)((char *)workspace + ((size_t)nb * NPAR * sizeof(float) + 255) / 256 * 256);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, theta_bf16, x, y, (long)n, (long)n, part, pl);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks(NPAR + 1, 256)), dim3(256), 0, s, (const float *)part,
                       (const float *)pl, (int)nb, (long)n, grad, loss);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CRK_OK : hip_err(e, "crk_mlp_loss_grad");
}

crk_status crk_mlp_adam(int64_t count, float *theta, float *m, float *v, const float *grad, double lr, double b1,
                        double b2, double eps, int t, uint16_t *theta_bf16, crk_stream stream)
{
    if (!theta || !m || !v || !grad || count < 1 || t < 1) { set_error(CRK_ERR_ARG, "bad argument"); return CRK_ERR_ARG; }
    const float c1 = (float)(1.0 - std::pow(b1, t)), c2 = (float)(1.0 - std::pow(b2, t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(count, 256)), dim3(256), 0, (hipStream_t)stream, (long)count, theta, m, v,
                       grad, (float)lr, (float)b1, (float)b2, (float)eps, c1, c2, theta_bf16);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CRK_OK : hip_err(e, "crk_mlp_adam");
}

crk_status crk_mlp_to_bf16(int64_t count, const float *theta, uint16_t *theta_bf16, crk_stream stream)
{
    if (!theta || !theta_bf16 || count < 1) { set_error(CRK_ERR_ARG, "bad argument"); return CRK_ERR_ARG; }
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(count, 256)), dim3(256), 0, (hipStream_t)stream, (long)count, theta,
                       theta_bf16);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CRK_OK : hip_err(e, "crk_mlp_to_bf16");
}

} // extern "C"
