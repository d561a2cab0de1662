// Source variants (rt_icosahedral_directions, rt_directional_directions).
//
// Section "Discrete model": an omnidirectional source emits N rays from its
// position along a uniform sampling of the unit sphere, icosahedron
// subdivision being one of the samplings named; for a directional source the
// sampling is made non-uniform (footnote).  Every ray keeps the energy 1/N,
// so a receiver's share n/N follows the directivity through the ray density.
//
// One thread per direction; FP64 without contraction, rounded once to FP32.
#include "common.h"

#include <cmath>

namespace rtac {
namespace {

struct IcoTables {
    double v[12][3];       // icosahedron vertices, unnormalised, edge 2
    int32_t edge[30][2];   // a < b, lexicographic
    int32_t face[20][3];   // a < b < c, lexicographic
};

// Direction g of the icosahedral grid of frequency f: the 12 vertices, then
// the f-1 inner points of each edge from a towards b, then the inner points
// (f-i-j) A + i B + j C of each face by i then j; pushed to the unit sphere.
__global__ void k_icosahedral(IcoTables T, int32_t f, int64_t n, float* __restrict__ dirs) {
#pragma clang fp contract(off)
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int64_t ne = f - 1;
    double x, y, z;
    if (g < 12) {
        x = T.v[g][0];
        y = T.v[g][1];
        z = T.v[g][2];
    } else if (g < 12 + 30 * ne) {
        const int64_t e = (g - 12) / ne, q = (g - 12) % ne + 1;
        const double* A = T.v[T.edge[e][0]];
        const double* B = T.v[T.edge[e][1]];
        const double wa = (double)(f - q), wb = (double)q;
        x = wa * A[0] + wb * B[0];
        y = wa * A[1] + wb * B[1];
        z = wa * A[2] + wb * B[2];
    } else {
        const int64_t nf = (int64_t)(f - 1) * (f - 2) / 2;   // inner points per face
        const int64_t r0 = g - 12 - 30 * ne;
        const int64_t t = r0 / nf, r = r0 % nf;
        // row i holds f-1-i points (j = 1 .. f-1-i); rows before row k+1 hold
        // S(k) = k (2f - 3 - k) / 2 points: take the k with S(k) <= r < S(k+1)
        const int64_t b = 2 * (int64_t)f - 3;
        int64_t k = (int64_t)(0.5 * ((double)b - sqrt((double)b * (double)b - 8.0 * (double)r)));
        k = k < 0 ? 0 : (k > f - 3 ? f - 3 : k);
        while (k > 0 && k * (b - k) / 2 > r) k--;
        while (k < f - 3 && (k + 1) * (b - k - 1) / 2 <= r) k++;
        const int64_t i = k + 1, j = r - k * (b - k) / 2 + 1;
        const double* A = T.v[T.face[t][0]];
        const double* B = T.v[T.face[t][1]];
        const double* C = T.v[T.face[t][2]];
        const double wa = (double)(f - i - j), wb = (double)i, wc = (double)j;
        x = wa * A[0] + wb * B[0] + wc * C[0];
        y = wa * A[1] + wb * B[1] + wc * C[1];
        z = wa * A[2] + wb * B[2] + wc * C[2];
    }
    const double nn = sqrt(x * x + y * y + z * z);
    dirs[3 * g] = (float)(x / nn);
    dirs[3 * g + 1] = (float)(y / nn);
    dirs[3 * g + 2] = (float)(z / nn);
}

struct Frame {
    double a[3], t1[3], t2[3];
};

// Direction i of n of the directional source: F = 1 - (2i+1)/(2n),
// z = 2 F^(1/(m+1)) - 1 (the inverse of the distribution ((1+z)/2)^(m+1) of
// cos theta under energy density (1 + cos theta)^m), phi = i pi (3 - sqrt5)
// mod 2 pi, in the frame (t1, t2, axis).
__global__ void k_directional(int64_t n, double inv_m1, Frame fr, float* __restrict__ dirs) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double pi = 3.14159265358979323846;
    const double golden = pi * (3.0 - sqrt(5.0));
    const double two_pi = 2.0 * pi;
    const double F = 1.0 - (double)(2 * i + 1) / (2.0 * (double)n);
    const double z = 2.0 * pow(F, inv_m1) - 1.0;
    const double phi = fmod((double)i * golden, two_pi);
    const double rho = sqrt(fmax(0.0, 1.0 - z * z));
    const double x = rho * cos(phi), y = rho * sin(phi);
    for (int c = 0; c < 3; c++) dirs[3 * i + c] = (float)(x * fr.t1[c] + y * fr.t2[c] + z * fr.a[c]);
}

IcoTables ico_tables() {
    IcoTables T{};
    const double phi = (1.0 + std::sqrt(5.0)) / 2.0;
    int k = 0;
    for (int place = 0; place < 3; place++)
        for (int sa = -1; sa <= 1; sa += 2)
            for (int sb = -1; sb <= 1; sb += 2) {
                const double a = (double)sa, b = (double)sb * phi;
                const double p[3][3] = {{0.0, a, b}, {a, b, 0.0}, {b, 0.0, a}};
                for (int c = 0; c < 3; c++) T.v[k][c] = p[place][c];
                k++;
            }
    bool adj[12][12];
    for (int p = 0; p < 12; p++)
        for (int q = 0; q < 12; q++) {
            double d2 = 0.0;
            for (int c = 0; c < 3; c++) d2 += (T.v[p][c] - T.v[q][c]) * (T.v[p][c] - T.v[q][c]);
            adj[p][q] = p != q && d2 < 4.5;
        }
    int ne = 0, nf = 0;
    for (int p = 0; p < 12; p++)
        for (int q = p + 1; q < 12; q++)
            if (adj[p][q]) {
                T.edge[ne][0] = p;
                T.edge[ne][1] = q;
                ne++;
            }
    for (int p = 0; p < 12; p++)
        for (int q = p + 1; q < 12; q++)
            for (int r = q + 1; r < 12; r++)
                if (adj[p][q] && adj[q][r] && adj[p][r]) {
                    T.face[nf][0] = p;
                    T.face[nf][1] = q;
                    T.face[nf][2] = r;
                    nf++;
                }
    return T;
}

}  // namespace
}  // namespace rtac

using namespace rtac;

extern "C" int rt_icosahedral_directions(int32_t f, float* dirs, void* stream) {
    RT_CHECK(f >= 1 && f <= 14000, RT_EINVAL, "rt_icosahedral_directions: frequency must be in [1, 14000]");
    RT_CHECK(dirs != nullptr, RT_EINVAL, "rt_icosahedral_directions: dirs is NULL");
    const int64_t n = 10 * (int64_t)f * f + 2;
    hipLaunchKernelGGL(k_icosahedral, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       ico_tables(), f, n, dirs);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" int rt_directional_directions(int64_t n, double m, const float* axis_host, float* dirs, void* stream) {
    RT_CHECK(n >= 0 && n < ((int64_t)1 << 31), RT_EINVAL, "rt_directional_directions: n out of range");
    RT_CHECK(std::isfinite(m) && m >= 0.0, RT_EINVAL, "rt_directional_directions: m must be finite and >= 0");
    RT_CHECK(axis_host != nullptr, RT_EINVAL, "rt_directional_directions: axis is NULL");
    double a[3] = {(double)axis_host[0], (double)axis_host[1], (double)axis_host[2]};
    const double an = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    RT_CHECK(std::isfinite(an) && an > 0.0, RT_EINVAL, "rt_directional_directions: axis must be finite, nonzero");
    if (n == 0) return RT_OK;
    RT_CHECK(dirs != nullptr, RT_EINVAL, "rt_directional_directions: dirs is NULL");
    Frame fr;
    for (int c = 0; c < 3; c++) fr.a[c] = a[c] / an;
    const double h[3] = {std::fabs(fr.a[0]) < 0.9 ? 1.0 : 0.0, std::fabs(fr.a[0]) < 0.9 ? 0.0 : 1.0, 0.0};
    const double ha = h[0] * fr.a[0] + h[1] * fr.a[1] + h[2] * fr.a[2];
    double t1[3];
    for (int c = 0; c < 3; c++) t1[c] = h[c] - ha * fr.a[c];
    const double tn = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    for (int c = 0; c < 3; c++) fr.t1[c] = t1[c] / tn;
    fr.t2[0] = fr.a[1] * fr.t1[2] - fr.a[2] * fr.t1[1];
    fr.t2[1] = fr.a[2] * fr.t1[0] - fr.a[0] * fr.t1[2];
    fr.t2[2] = fr.a[0] * fr.t1[1] - fr.a[1] * fr.t1[0];
    hipLaunchKernelGGL(k_directional, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n,
                       1.0 / (m + 1.0), fr, dirs);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
