// Input padding: an instance with n_u below the matrix-core tile (n_x = 16 or
// 32, n_u < 16) is solved as the equivalent problem with n_u = 16, whose
// extra inputs act on nothing: B gets zero columns, Q_xw zero columns, Q_w an
// identity block and l_w zeros.  Those inputs are decoupled from the rest and
// strictly convex, so their optimal value is 0, and x, lam, the optimal value
// and the first n_u inputs are those of the caller's problem (Sec. 2: P(N) is
// a UFTOC problem of any input dimension).  k_pad writes the padded arrays
// into the workspace before a call, k_unpad copies w back after it.
#include <hip/hip_runtime.h>

#include "rs_launch.hpp"

namespace rs {
namespace pad {

constexpr int NT = 256;
constexpr int YB = 8;            // blocks per instance (grid y); each strides over the stages

__global__ void __launch_bounds__(NT) k_pad(const PadArgs *args) {
    const PadArgs a = args[blockIdx.x];
    if (a.flags & PROB_SKIP) return;
    const int nx = a.nx, nu = a.nu, np = a.nup, tid = threadIdx.x;
    for (int t = blockIdx.y; t < a.N; t += gridDim.y) {
        if (t == 0 || a.sB) {
            const double *B = a.B + (int64_t)t * a.sB;
            double *Bp = a.Bp + (int64_t)t * a.sBp;
            for (int e = tid; e < nx * np; e += NT) {
                const int i = e / np, j = e - (e / np) * np;
                Bp[e] = j < nu ? B[i * nu + j] : 0.0;
            }
        }
        if (t == 0 || a.sQw) {
            const double *Q = a.Qw + (int64_t)t * a.sQw;
            double *Qp = a.Qwp + (int64_t)t * a.sQwp;
            for (int e = tid; e < np * np; e += NT) {
                const int i = e / np, j = e - (e / np) * np;
                Qp[e] = (i < nu && j < nu) ? Q[i * nu + j] : (i == j ? 1.0 : 0.0);
            }
        }
        if (a.Qxw && (t == 0 || a.sQxw)) {
            const double *S = a.Qxw + (int64_t)t * a.sQxw;
            double *Sp = a.Qxwp + (int64_t)t * a.sQxwp;
            for (int e = tid; e < nx * np; e += NT) {
                const int i = e / np, j = e - (e / np) * np;
                Sp[e] = j < nu ? S[i * nu + j] : 0.0;
            }
        }
        if (a.lw && (t == 0 || a.slw)) {
            const double *l = a.lw + (int64_t)t * a.slw;
            double *lp = a.lwp + (int64_t)t * a.slwp;
            for (int j = tid; j < np; j += NT) lp[j] = j < nu ? l[j] : 0.0;
        }
    }
}

__global__ void __launch_bounds__(NT) k_unpad(const PadArgs *args) {
    const PadArgs a = args[blockIdx.x];
    if (a.flags & PROB_SKIP) return;
    const int nu = a.nu, np = a.nup;
    for (int t = blockIdx.y; t < a.N; t += gridDim.y)
        for (int j = threadIdx.x; j < nu; j += NT) a.w[(int64_t)t * nu + j] = a.wp[(int64_t)t * np + j];
}

}  // namespace pad

hipError_t launch_pad(const PadArgs *args, int npad, bool back, hipStream_t st) {
    if (npad < 1) return hipSuccess;
    if (back)
        hipLaunchKernelGGL(pad::k_unpad, dim3(npad, pad::YB), dim3(pad::NT), 0, st, args);
    else
        hipLaunchKernelGGL(pad::k_pad, dim3(npad, pad::YB), dim3(pad::NT), 0, st, args);
    return hipGetLastError();
}

}  // namespace rs
