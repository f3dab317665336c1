// Polar-cap reorientation of a map (Sec. 4, Conclusions: survey maps rotated
// onto a polar cap keep the number of rings a ring-based convolution touches
// small).  A rotated copy is resampled at the nearest pixel: output pixel p,
// with centre n_p, takes the input pixel containing R^T n_p, so a feature at
// direction c of the input appears at R c of the output.  Geometry and point
// location run in FP64 (HEALPix RING scheme, Gorski et al. 2005).
#include <cmath>
#include <string>

#include "arkcos_internal.hpp"

namespace arkcos {

struct Rot {
    double r[9];   // row-major
};

// The RING pixel containing the direction (z = cos theta, phi).  With
// t = phi / (pi/2) in [0, 4): in the equatorial zone |z| <= 2/3 the pixel
// boundaries are the lines N (1/2 + t -+ 3z/4) = integer, and the two
// integer parts a, b give the ring N + a - b and the in-ring index
// (a + b - N + [ring - N odd] + 1) / 2; in the caps, with
// s = N sqrt(3 (1 - |z|)) and tq the longitude within its quadrant, the
// boundaries are tq s = integer and (1 - tq) s = integer, and the ring from
// the nearest pole is their integer parts' sum + 1.  Contraction into FMAs is
// off, so each product is rounded as written.
__device__ __forceinline__ long long ring_pixel_of(int N, double z, double phi)
{
#pragma clang fp contract(off)
    const double dN = (double)N;
    double t = phi / (0.5 * M_PI);
    t = fmod(t, 4.0);
    if (t < 0.0) t += 4.0;
    if (fabs(z) <= 2.0 / 3.0) {
        const long long a = (long long)floor(dN * (0.5 + t - 0.75 * z));
        const long long b = (long long)floor(dN * (0.5 + t + 0.75 * z));
        const long long ir = (long long)N + 1 + a - b;   // ring N + ir - 1
        const long long shift = (ir & 1) ? 0 : 1;
        long long ip = (a + b - N + shift + 1) / 2;
        const long long nr = 4LL * N;
        ip %= nr;
        if (ip < 0) ip += nr;
        return 2LL * N * (N - 1) + nr * (ir - 1) + ip;
    }
    const double tq = t - floor(t);
    const double sr = dN * sqrt(3.0 * (1.0 - fabs(z)));
    long long k = (long long)floor(tq * sr) + (long long)floor((1.0 - tq) * sr) + 1;
    k = k > N ? N : (k < 1 ? 1 : k);   // k = N only beside |z| = 2/3
    long long ip = (long long)floor(t * (double)k);
    ip %= 4 * k;
    if (z > 0.0) return 2 * k * (k - 1) + ip;
    return 12LL * N * N - 2 * k * (k + 1) + ip;
}

// One workgroup per output ring of the range.
__global__ __launch_bounds__(256) void k_rotate(int N, Rot R, const float *__restrict__ in,
                                                float *__restrict__ out, int nbatch, int ring0)
{
#pragma clang fp contract(off)
    const int i = ring0 + (int)blockIdx.x;   // 1-based ring
    const double dN = (double)N;
    double z, s, phi0;
    long long n, first;
    if (i < N) {
        const double a = (double)i * (double)i / (3.0 * dN * dN);
        z = 1.0 - a;
        s = sqrt(a * (2.0 - a));
        n = 4LL * i;
        first = 2LL * i * (i - 1);
        phi0 = 0.5 * M_PI / (2.0 * (double)i);
    } else if (i <= 3 * N) {
        z = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * dN);
        s = sqrt((1.0 - z) * (1.0 + z));
        n = 4LL * N;
        first = 2LL * N * (N - 1) + 4LL * N * (i - N);
        phi0 = ((i - N) % 2 == 0) ? 0.5 * M_PI / (2.0 * dN) : 0.0;
    } else {
        const long long k = 4LL * N - i;
        const double a = (double)k * (double)k / (3.0 * dN * dN);
        z = a - 1.0;
        s = sqrt(a * (2.0 - a));
        n = 4 * k;
        first = 12LL * N * N - 2 * k * (k + 1);
        phi0 = 0.5 * M_PI / (2.0 * (double)k);
    }
    const double dphi = 2.0 * M_PI / (double)n;
    const long long npix = 12LL * N * N;
    for (long long j = threadIdx.x; j < n; j += blockDim.x) {
        const double phi = phi0 + (double)j * dphi;
        const double v0 = s * cos(phi), v1 = s * sin(phi), v2 = z;
        double w[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) w[c] = R.r[c] * v0 + R.r[3 + c] * v1 + R.r[6 + c] * v2;
        const double rr = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        const long long q = ring_pixel_of(N, w[2] / rr, atan2(w[1], w[0]));
        for (int b = 0; b < nbatch; ++b) out[b * npix + first + j] = in[b * npix + q];
    }
}

static int check_rotation(const double *r)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double d = 0.0;
            for (int k = 0; k < 3; ++k) d += r[a * 3 + k] * r[b * 3 + k];
            if (!(std::fabs(d - (a == b ? 1.0 : 0.0)) <= 1e-9))
                return fail(ARKCOS_EINVAL, "rot is not orthonormal (|R R^T - I| > 1e-9)");
        }
    const double det = r[0] * (r[4] * r[8] - r[5] * r[7]) - r[1] * (r[3] * r[8] - r[5] * r[6]) +
                       r[2] * (r[3] * r[7] - r[4] * r[6]);
    if (!(det > 0.0)) return fail(ARKCOS_EINVAL, "rot is a reflection (det < 0)");
    return ARKCOS_OK;
}

}  // namespace arkcos

using namespace arkcos;

extern "C" {

int arkcos_rotation_to_pole(double theta, double phi, double *rot)
{
    clear_error();
    if (!rot) return fail(ARKCOS_EINVAL, "NULL pointer");
    if (!std::isfinite(theta) || !std::isfinite(phi))
        return fail(ARKCOS_EINVAL, "theta and phi must be finite");
    // R_y(-theta) R_z(-phi): (theta, phi) -> longitude 0 -> the pole
    const double ct = std::cos(theta), st = std::sin(theta);
    const double cp = std::cos(phi), sp = std::sin(phi);
    const double m[9] = {ct * cp, ct * sp, -st, -sp, cp, 0.0, st * cp, st * sp, ct};
    for (int k = 0; k < 9; ++k) rot[k] = m[k];
    return ARKCOS_OK;
}

int arkcos_rotate_map(int nside, const double *rot, const float *d_in, float *d_out, int nbatch,
                      int ring_first, int ring_last, void *stream)
{
    clear_error();
    TraceRange tr("arkcos_rotate_map");
    if (!rot || !d_in || !d_out) return fail(ARKCOS_EINVAL, "NULL pointer");
    if (nside < 1 || nside > ARKCOS_MAX_NSIDE)
        return fail(ARKCOS_EINVAL, "nside must lie in 1.." + std::to_string(ARKCOS_MAX_NSIDE));
    if (nbatch < 1) return fail(ARKCOS_EINVAL, "nbatch must be >= 1");
    if (ring_first == 0 && ring_last == 0) {
        ring_first = 1;
        ring_last = 4 * nside - 1;
    }
    if (!(ring_first >= 1 && ring_first <= ring_last && ring_last <= 4 * nside - 1))
        return fail(ARKCOS_EINVAL, "ring range must be 0, 0 or 1 <= ring_first <= ring_last <= "
                                   "4 nside - 1");
    int rc = check_rotation(rot);
    if (rc) return rc;
    const size_t bytes = (size_t)nbatch * 12 * (size_t)nside * (size_t)nside * sizeof(float);
    const char *a = reinterpret_cast<const char *>(d_in);
    const char *b = reinterpret_cast<const char *>(d_out);
    if (a < b + bytes && b < a + bytes) return fail(ARKCOS_EINVAL, "d_in and d_out overlap");
    Rot R;
    for (int k = 0; k < 9; ++k) R.r[k] = rot[k];
    hipLaunchKernelGGL(k_rotate, dim3(ring_last - ring_first + 1), dim3(256), 0,
                       (hipStream_t)stream, nside, R, d_in, d_out, nbatch, ring_first);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

}  // extern "C"
