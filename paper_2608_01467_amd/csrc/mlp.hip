// mlp.hip -- the learned cost model's network: inference, gradients and the
// optimiser step as gfx950 kernels (C ABI in include/fhs.h).
//
// Network (FP64): x (n_in) -> tanh(W1 x + b1) -> tanh(W2 a1 + b2) -> w3.a2 + b3.
// Flat parameters, in order: W1 [h1][n_in], b1 [h1], W2 [h2][h1], b2 [h2],
// w3 [h2], b3.  Loss: mean squared error over the batch.  Optimiser: Adam
// (Kingma & Ba 2015).  Sizes are tiny (n_in, h1, h2 <= 64, batches of a few
// thousand rows), so each workgroup takes a tile of samples, keeps the tile's
// activations in LDS and one thread per hidden unit; gradients are summed per
// tile and then across tiles in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/fhs.h"

namespace fhs {
namespace {

constexpr int kTile = 16;      // samples per workgroup
constexpr int kMaxUnits = 64;  // max n_in, h1, h2
constexpr int kThreads = 64;

struct Shape {
    int n_in, h1, h2;
};

__host__ __device__ inline size_t n_params(const Shape &s) {
    return static_cast<size_t>(s.h1) * s.n_in + s.h1 + static_cast<size_t>(s.h2) * s.h1 + s.h2 +
           s.h2 + 1;
}

struct Offsets {
    size_t W1, b1, W2, b2, w3, b3;
};

__host__ __device__ inline Offsets offsets(const Shape &s) {
    Offsets o;
    o.W1 = 0;
    o.b1 = o.W1 + static_cast<size_t>(s.h1) * s.n_in;
    o.W2 = o.b1 + s.h1;
    o.b2 = o.W2 + static_cast<size_t>(s.h2) * s.h1;
    o.w3 = o.b2 + s.h2;
    o.b3 = o.w3 + s.h2;
    return o;
}

// Forward pass of a tile; activations stay in LDS for the caller.
__device__ void tile_forward(const Shape &sh, const double *__restrict__ p,
                             const double *__restrict__ x, uint32_t s0, uint32_t ns,
                             double (*sx)[kMaxUnits], double (*a1)[kMaxUnits],
                             double (*a2)[kMaxUnits], double *y) {
    const Offsets o = offsets(sh);
    const int t = threadIdx.x;
    for (int i = t; i < kTile * sh.n_in; i += blockDim.x) {
        const int s = i / sh.n_in, k = i % sh.n_in;
        sx[s][k] = (static_cast<uint32_t>(s) < ns) ? x[static_cast<size_t>(s0 + s) * sh.n_in + k] : 0.0;
    }
    __syncthreads();
    for (int j = t; j < sh.h1; j += blockDim.x) {
        for (int s = 0; s < kTile; ++s) {
            double z = p[o.b1 + j];
            for (int k = 0; k < sh.n_in; ++k) z = fma(p[o.W1 + static_cast<size_t>(j) * sh.n_in + k], sx[s][k], z);
            a1[s][j] = tanh(z);
        }
    }
    __syncthreads();
    for (int j = t; j < sh.h2; j += blockDim.x) {
        for (int s = 0; s < kTile; ++s) {
            double z = p[o.b2 + j];
            for (int k = 0; k < sh.h1; ++k) z = fma(p[o.W2 + static_cast<size_t>(j) * sh.h1 + k], a1[s][k], z);
            a2[s][j] = tanh(z);
        }
    }
    __syncthreads();
    if (t < kTile) {
        double z = p[o.b3];
        for (int j = 0; j < sh.h2; ++j) z = fma(p[o.w3 + j], a2[t][j], z);
        y[t] = z;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_mlp_forward(Shape sh, const double *p, const double *x,
                                                          uint32_t B, double *y, double *act) {
    __shared__ double sx[kTile][kMaxUnits], a1[kTile][kMaxUnits], a2[kTile][kMaxUnits];
    __shared__ double sy[kTile];
    const uint32_t s0 = blockIdx.x * kTile;
    const uint32_t ns = min(static_cast<uint32_t>(kTile), B - s0);
    tile_forward(sh, p, x, s0, ns, sx, a1, a2, sy);
    const int t = threadIdx.x;
    if (static_cast<uint32_t>(t) < ns) y[s0 + t] = sy[t];
    if (act) {
        const int w = sh.h1 + sh.h2;
        for (int i = t; i < static_cast<int>(ns) * w; i += blockDim.x) {
            const int s = i / w, k = i % w;
            act[static_cast<size_t>(s0 + s) * w + k] = k < sh.h1 ? a1[s][k] : a2[s][k - sh.h1];
        }
    }
}

// Per-tile gradient partials of the mean squared error, plus the tile's
// share of the loss, written to part[tile][n_params + 1].
__global__ __launch_bounds__(kThreads) void k_mlp_backward(Shape sh, const double *p, const double *x,
                                                           const double *tgt, uint32_t B,
                                                           double *part) {
    __shared__ double sx[kTile][kMaxUnits], a1[kTile][kMaxUnits], a2[kTile][kMaxUnits];
    __shared__ double sy[kTile], dy[kTile];
    __shared__ double dz1[kTile][kMaxUnits], dz2[kTile][kMaxUnits];
    const Offsets o = offsets(sh);
    const size_t np = n_params(sh);
    const uint32_t s0 = blockIdx.x * kTile;
    const uint32_t ns = min(static_cast<uint32_t>(kTile), B - s0);
    const int t = threadIdx.x;
    tile_forward(sh, p, x, s0, ns, sx, a1, a2, sy);
    if (t < kTile) {
        const bool live = static_cast<uint32_t>(t) < ns;
        dy[t] = live ? 2.0 * (sy[t] - tgt[s0 + t]) / static_cast<double>(B) : 0.0;
    }
    __syncthreads();
    for (int j = t; j < sh.h2; j += blockDim.x)
        for (int s = 0; s < kTile; ++s) dz2[s][j] = dy[s] * p[o.w3 + j] * (1.0 - a2[s][j] * a2[s][j]);
    __syncthreads();
    for (int k = t; k < sh.h1; k += blockDim.x)
        for (int s = 0; s < kTile; ++s) {
            double g = 0.0;
            for (int j = 0; j < sh.h2; ++j) g = fma(p[o.W2 + static_cast<size_t>(j) * sh.h1 + k], dz2[s][j], g);
            dz1[s][k] = g * (1.0 - a1[s][k] * a1[s][k]);
        }
    __syncthreads();
    double *out = part + static_cast<size_t>(blockIdx.x) * (np + 1);
    for (int j = t; j < sh.h1; j += blockDim.x) {
        for (int k = 0; k < sh.n_in; ++k) {
            double g = 0.0;
            for (int s = 0; s < kTile; ++s) g = fma(dz1[s][j], sx[s][k], g);
            out[o.W1 + static_cast<size_t>(j) * sh.n_in + k] = g;
        }
        double gb = 0.0;
        for (int s = 0; s < kTile; ++s) gb += dz1[s][j];
        out[o.b1 + j] = gb;
    }
    for (int j = t; j < sh.h2; j += blockDim.x) {
        for (int k = 0; k < sh.h1; ++k) {
            double g = 0.0;
            for (int s = 0; s < kTile; ++s) g = fma(dz2[s][j], a1[s][k], g);
            out[o.W2 + static_cast<size_t>(j) * sh.h1 + k] = g;
        }
        double gb = 0.0, gw = 0.0;
        for (int s = 0; s < kTile; ++s) {
            gb += dz2[s][j];
            gw = fma(dy[s], a2[s][j], gw);
        }
        out[o.b2 + j] = gb;
        out[o.w3 + j] = gw;
    }
    if (t == 0) {
        double gb = 0.0, l = 0.0;
        for (int s = 0; s < static_cast<int>(ns); ++s) {
            gb += dy[s];
            const double d = sy[s] - tgt[s0 + s];
            l = fma(d, d, l);
        }
        out[o.b3] = gb;
        out[np] = l / static_cast<double>(B);
    }
}

// grad[i] = sum over tiles, in tile order; the last slot is the loss.
__global__ void k_mlp_reduce(const double *part, uint32_t tiles, size_t np, double *grad,
                             double *loss) {
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i > np) return;
    double g = 0.0;
    for (uint32_t k = 0; k < tiles; ++k) g += part[static_cast<size_t>(k) * (np + 1) + i];
    if (i < np) grad[i] = g;
    else if (loss) *loss = g;
}

__global__ void k_mlp_adam(size_t n, double *p, const double *g, double *m, double *v, double lr,
                           double b1, double b2, double eps, double c1, double c2) {
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrt(vi * c2) + eps);
}

bool shape_ok(const fhs_mlp_shape *s) {
    return s && s->n_in >= 1 && s->h1 >= 1 && s->h2 >= 1 && s->n_in <= kMaxUnits &&
           s->h1 <= kMaxUnits && s->h2 <= kMaxUnits;
}

Shape to_shape(const fhs_mlp_shape *s) {
    return Shape{static_cast<int>(s->n_in), static_cast<int>(s->h1), static_cast<int>(s->h2)};
}

}  // namespace

hipError_t mlp_forward(const fhs_mlp_shape *s, const double *p, const double *x, uint32_t B,
                       double *y, double *act, hipStream_t st) {
    const uint32_t tiles = (B + kTile - 1) / kTile;
    k_mlp_forward<<<tiles, kThreads, 0, st>>>(to_shape(s), p, x, B, y, act);
    return hipGetLastError();
}

}  // namespace fhs

using namespace fhs;

extern "C" fhs_status fhs_mlp_param_count(const fhs_mlp_shape *s, size_t *n) {
    if (!shape_ok(s) || !n) return FHS_EINVAL;
    *n = n_params(to_shape(s));
    return FHS_OK;
}

extern "C" fhs_status fhs_mlp_workspace_size(const fhs_mlp_shape *s, uint32_t B, size_t *bytes) {
    if (!shape_ok(s) || !bytes || B == 0) return FHS_EINVAL;
    const size_t tiles = (B + kTile - 1) / kTile;
    *bytes = tiles * (n_params(to_shape(s)) + 1) * sizeof(double);
    return FHS_OK;
}

extern "C" fhs_status fhs_mlp_forward(const fhs_mlp_shape *s, const double *d_params,
                                      const double *d_x, uint32_t B, double *d_y, double *d_act,
                                      void *stream) {
    if (!shape_ok(s) || !d_params || !d_x || !d_y) return FHS_EINVAL;
    if (B == 0) return FHS_OK;
    return mlp_forward(s, d_params, d_x, B, d_y, d_act, static_cast<hipStream_t>(stream)) == hipSuccess
               ? FHS_OK
               : FHS_EHIP;
}

extern "C" fhs_status fhs_mlp_backward(const fhs_mlp_shape *s, const double *d_params,
                                       const double *d_x, const double *d_t, uint32_t B,
                                       double *d_grad, double *d_loss, void *d_ws, size_t ws_bytes,
                                       void *stream) {
    if (!shape_ok(s) || !d_params || !d_x || !d_t || !d_grad || B == 0) return FHS_EINVAL;
    size_t need = 0;
    fhs_mlp_workspace_size(s, B, &need);
    if (!d_ws || ws_bytes < need) return FHS_ENOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Shape sh = to_shape(s);
    const uint32_t tiles = (B + kTile - 1) / kTile;
    double *part = static_cast<double *>(d_ws);
    k_mlp_backward<<<tiles, kThreads, 0, st>>>(sh, d_params, d_x, d_t, B, part);
    const size_t np = n_params(sh);
    k_mlp_reduce<<<static_cast<uint32_t>((np + 1 + 255) / 256), 256, 0, st>>>(part, tiles, np, d_grad,
                                                                               d_loss);
    return hipGetLastError() == hipSuccess ? FHS_OK : FHS_EHIP;
}

extern "C" fhs_status fhs_mlp_adam(size_t n, double *d_params, const double *d_grad, double *d_m,
                                   double *d_v, uint32_t step, double lr, double beta1, double beta2,
                                   double eps, void *stream) {
    if (!d_params || !d_grad || !d_m || !d_v || step == 0 || !(lr > 0.0) || !(beta1 >= 0.0) ||
        !(beta1 < 1.0) || !(beta2 >= 0.0) || !(beta2 < 1.0) || !(eps >= 0.0))
        return FHS_EINVAL;
    if (n == 0) return FHS_OK;
    const double c1 = 1.0 / (1.0 - std::pow(beta1, static_cast<double>(step)));
    const double c2 = 1.0 / (1.0 - std::pow(beta2, static_cast<double>(step)));
    k_mlp_adam<<<static_cast<uint32_t>((n + 255) / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(
        n, d_params, d_grad, d_m, d_v, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? FHS_OK : FHS_EHIP;
}
