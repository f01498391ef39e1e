// Akima spline motion model of the motion-estimation experiment (Sec.
// "Optimization"): every rigid parameter of T(theta) along the scan follows
// an Akima spline (Akima 1970) through a few nodes, and the optimiser works
// on the node values.  Two kernels: node values -> per-view parameters, and
// the chain rule from d cost / d theta back to the nodes.  FP64 throughout;
// the node derivative comes from one forward-mode dual per (hypothesis,
// parameter, node), summed over the views it influences in view order
// (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include "ecc_internal.hpp"
#include "projective.hpp"

namespace ecc {

namespace {

__device__ __forceinline__ double s_abs(double x) { return fabs(x); }
__device__ __forceinline__ Dual s_abs(Dual x) { return x.v < 0.0 ? -x : x; }

// Node values are read through an accessor y(i) (a node value, or a dual
// number carrying d/d node j) rather than a per-thread array: an Akima value
// needs only the six nodes around its segment.

// Segment slope m_k for k in [-2, n]: interior slopes from the nodes, two
// linearly extrapolated slopes beyond each end.
template <class T, class Y>
__device__ T seg_slope(const SplineKnots &kn, const Y &y, int k) {
    const int n = kn.n;
    auto m = [&](int i) { return (y(i + 1) - y(i)) / T(kn.x[i + 1] - kn.x[i]); };
    if (k >= 0 && k <= n - 2) return m(k);
    if (k == -1) return T(2.0) * m(0) - m(1);
    if (k == -2) return T(3.0) * m(0) - T(2.0) * m(1);  // 2 m_{-1} - m_0
    if (k == n - 1) return T(2.0) * m(n - 2) - m(n - 3);
    return T(3.0) * m(n - 2) - T(2.0) * m(n - 3);  // k == n: 2 m_{n-1} - m_{n-2}
}

// Akima's derivative estimate at node i.
template <class T, class Y>
__device__ T node_slope(const SplineKnots &kn, const Y &y, int i) {
    const T m_2 = seg_slope<T>(kn, y, i - 2), m_1 = seg_slope<T>(kn, y, i - 1);
    const T m0 = seg_slope<T>(kn, y, i), m1 = seg_slope<T>(kn, y, i + 1);
    const T w_hi = s_abs(m1 - m0), w_lo = s_abs(m_1 - m_2);
    if (g_val(w_hi) + g_val(w_lo) == 0.0) return T(0.5) * (m_1 + m0);
    return (w_hi * m_1 + w_lo * m0) / (w_hi + w_lo);
}

__device__ int segment_of(const SplineKnots &kn, double x) {
    int i = 0;
    while (i < kn.n - 2 && x >= kn.x[i + 1]) ++i;
    return i;
}

// The interpolant at x (inside [x_0, x_{n-1}]).
template <class T, class Y>
__device__ T akima_at(const SplineKnots &kn, const Y &y, double x) {
    const int i = segment_of(kn, x);
    const double h = kn.x[i + 1] - kn.x[i];
    const double s = (x - kn.x[i]) / h, s2 = s * s, s3 = s2 * s;
    const T ti = node_slope<T>(kn, y, i), ti1 = node_slope<T>(kn, y, i + 1);
    return T(2 * s3 - 3 * s2 + 1) * y(i) + T((s3 - 2 * s2 + s) * h) * ti + T(-2 * s3 + 3 * s2) * y(i + 1) +
           T((s3 - s2) * h) * ti1;
}

// thread = (hypothesis, view, parameter)
__global__ __launch_bounds__(256) void spline_motion_kernel(SplineKnots kn, int B, int n_views,
                                                            const double *__restrict__ nodes,
                                                            double *__restrict__ theta) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * n_views * 6) return;
    const int c = (int)(idx % 6);
    const int64_t bl = idx / 6;
    const int lam = (int)(bl % n_views), b = (int)(bl / n_views);
    const double *yb = nodes + ((int64_t)b * 6 + c) * kn.n;
    auto y = [yb](int i) { return yb[i]; };
    theta[idx] = akima_at<double>(kn, y, (double)lam);
}

// workgroup = (hypothesis, parameter, node): sum over the views the node
// influences (segments j - 3 .. j + 2) of grad_theta * d theta / d y_j, the
// views dealt over the 256 threads and the partial sums added in a fixed tree
// order.
__global__ __launch_bounds__(256) void spline_grad_kernel(SplineKnots kn, int B, int n_views,
                                                          const double *__restrict__ nodes,
                                                          const float *__restrict__ grad_theta,
                                                          double *__restrict__ grad_nodes) {
    const int64_t idx = blockIdx.x;  // the grid holds exactly B * 6 * n workgroups
    const int j = (int)(idx % kn.n);
    const int64_t bc = idx / kn.n;
    const int c = (int)(bc % 6), b = (int)(bc / 6);
    const double *yb = nodes + bc * kn.n;
    auto y = [yb, j](int i) { return Dual(yb[i], i == j ? 1.0 : 0.0); };
    const double x_lo = kn.x[j >= 3 ? j - 3 : 0], x_hi = kn.x[j + 3 <= kn.n - 1 ? j + 3 : kn.n - 1];
    int l0 = (int)ceil(x_lo), l1 = (int)floor(x_hi);
    if (l0 < 0) l0 = 0;
    if (l1 > n_views - 1) l1 = n_views - 1;
    double acc = 0.0;
    for (int lam = l0 + (int)threadIdx.x; lam <= l1; lam += blockDim.x)
        acc += (double)grad_theta[((int64_t)b * n_views + lam) * 6 + c] * akima_at<Dual>(kn, y, (double)lam).d;
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad_nodes[idx] = red[0];
}

}  // namespace

hipError_t launch_spline_motion(const SplineKnots &kn, int B, int n_views, const double *nodes, double *theta,
                                hipStream_t s) {
    const int64_t n = (int64_t)B * n_views * 6;
    hipLaunchKernelGGL(spline_motion_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, kn, B, n_views,
                       nodes, theta);
    return hipGetLastError();
}

hipError_t launch_spline_grad(const SplineKnots &kn, int B, int n_views, const double *nodes,
                              const float *grad_theta, double *grad_nodes, hipStream_t s) {
    const int64_t n = (int64_t)B * 6 * kn.n;
    hipLaunchKernelGGL(spline_grad_kernel, dim3((unsigned)n), dim3(256), 0, s, kn, B, n_views, nodes, grad_theta,
                       grad_nodes);
    return hipGetLastError();
}

}  // namespace ecc
