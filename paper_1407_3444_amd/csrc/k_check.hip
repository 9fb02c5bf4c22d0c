// k_check.hip -- the content scan of a call's device inputs (Sec. II takes band energies and
// normalised eigenvectors on the mesh as the method's inputs): non-finite values in the band
// energies, eigenvector coefficients and frequencies, and eigenvectors whose squared norm differs
// from one.  The verdict is a bit mask OR-ed into one word of the caller's workspace; the host
// copies it out asynchronously.  The scans read each array once (HBM-bound, a few hundred
// microseconds for the largest inputs) and never stop the computation that follows.
#include "chi0_internal.h"

namespace chi0 {

namespace {

constexpr int kScanThreads = 256;

__global__ __launch_bounds__(kScanThreads) void clear_flag_kernel(unsigned *flag) { *flag = 0u; }

// Every element of a float64 array finite; bit set otherwise.  One wave-level ballot per block
// of loads, so a bad array costs one atomic per wave rather than one per element.
__global__ __launch_bounds__(kScanThreads) void scan_finite_kernel(const double *__restrict__ p, int64_t n,
                                                                  unsigned bit, unsigned *flag)
{
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        bad |= !isfinite(p[i]);
    if (__ballot(bad) != 0ull && (threadIdx.x & (kWave - 1)) == 0) atomicOr(flag, bit);
}

// Eigenvectors c[Nk][no][nb] (complex, interleaved): thread (k, n) sums |c_{o,n}(k)|^2 over o;
// consecutive threads take consecutive bands of one k, so each orbital row is read coalesced.
__global__ __launch_bounds__(kScanThreads) void scan_eigvec_kernel(const double *__restrict__ c, int64_t nk, int no,
                                                                  int nb, unsigned bit_nonfinite, unsigned bit_norm,
                                                                  double tol, unsigned *flag)
{
    unsigned bits = 0u;
    const int64_t total = nk * nb;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int64_t k = t / nb;
        const int n = (int)(t - k * nb);
        const double *col = c + 2 * (k * no * (int64_t)nb + n);
        double s = 0.0;
        for (int o = 0; o < no; ++o) {
            const double re = col[2 * (int64_t)o * nb], im = col[2 * (int64_t)o * nb + 1];
            s = fma(re, re, fma(im, im, s));
        }
        if (!isfinite(s)) bits |= bit_nonfinite;
        else if (!(fabs(s - 1.0) <= tol)) bits |= bit_norm;
    }
    const bool any = bits != 0u;
    if (__ballot(any) != 0ull) {
        if (any) atomicOr(flag, bits);
    }
}

// Large bases (plane waves, thousands of coefficients per eigenvector): one workgroup per k, so
// the serial loop over orbitals of the kernel above does not leave HBM idle.  Thread j takes band
// n = j % nb and the orbitals o = og, og + G, ... with og = j / nb (G = kScanThreads / nb groups);
// consecutive threads read consecutive coefficients of the k's [no][nb] block.  The G partial sums
// of each band are added in LDS in a fixed order.
__global__ __launch_bounds__(kScanThreads) void scan_eigvec_wide_kernel(const double *__restrict__ c, int64_t nk,
                                                                       int no, int nb, unsigned bit_nonfinite,
                                                                       unsigned bit_norm, double tol, unsigned *flag)
{
    __shared__ double part[kScanThreads];
    const int j = threadIdx.x;
    const int G = kScanThreads / nb;
    const int og = j / nb, n = j - og * nb;
    unsigned bits = 0u;
    for (int64_t k = blockIdx.x; k < nk; k += gridDim.x) {
        double s0 = 0.0, s1 = 0.0;
        if (og < G) {
            const double *base = c + 2 * (k * no * (int64_t)nb + n);
            int o = og;
            for (; o + G < no; o += 2 * G) {
                const double2 a = *reinterpret_cast<const double2 *>(base + 2 * (int64_t)o * nb);
                const double2 b = *reinterpret_cast<const double2 *>(base + 2 * (int64_t)(o + G) * nb);
                s0 = fma(a.x, a.x, fma(a.y, a.y, s0));
                s1 = fma(b.x, b.x, fma(b.y, b.y, s1));
            }
            if (o < no) {
                const double2 a = *reinterpret_cast<const double2 *>(base + 2 * (int64_t)o * nb);
                s0 = fma(a.x, a.x, fma(a.y, a.y, s0));
            }
        }
        part[j] = s0 + s1;
        __syncthreads();
        if (j < nb) {
            double s = 0.0;
            for (int g = 0; g < G; ++g) s += part[g * nb + j];
            if (!isfinite(s)) bits |= bit_nonfinite;
            else if (!(fabs(s - 1.0) <= tol)) bits |= bit_norm;
        }
        __syncthreads();
    }
    const bool any = bits != 0u;
    if (__ballot(any) != 0ull) {
        if (any) atomicOr(flag, bits);
    }
}

int scan_blocks(int64_t n)
{
    const int64_t b = (n + kScanThreads - 1) / kScanThreads;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

hipError_t launch_scan_clear(unsigned *flag, hipStream_t s)
{
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
    return hipGetLastError();
}

hipError_t launch_scan_finite(const double *p, int64_t n, unsigned bit, unsigned *flag, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scan_finite_kernel, dim3(scan_blocks(n)), dim3(kScanThreads), 0, s, p, n, bit, flag);
    return hipGetLastError();
}

hipError_t launch_scan_eigvec(const double *c, int64_t nk, int no, int nb, unsigned bit_nonfinite, unsigned bit_norm,
                              double tol, unsigned *flag, hipStream_t s)
{
    if (nk <= 0 || no <= 0 || nb <= 0) return hipSuccess;
    if (no > kMaxOrbSmall && nb <= kScanThreads) {
        const unsigned nblk = (unsigned)(nk < 65536 ? nk : 65536);
        hipLaunchKernelGGL(scan_eigvec_wide_kernel, dim3(nblk), dim3(kScanThreads), 0, s, c, nk, no, nb, bit_nonfinite,
                           bit_norm, tol, flag);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(scan_eigvec_kernel, dim3(scan_blocks(nk * nb)), dim3(kScanThreads), 0, s, c, nk, no, nb,
                       bit_nonfinite, bit_norm, tol, flag);
    return hipGetLastError();
}

}  // namespace chi0
