// kernels_demag.hip -- the demagnetising kernel, built in FP64 on the GPU.
//
// Section "Magnetostatic field", paragraph "Magnetostatic kernel": the field of
// a uniformly magnetised cell, averaged over the destination cell.  For every
// displacement d = (i dx, j dy, k dz) of the non-negative octant:
//   near (|d| < 2.5 cell diagonals): the closed form of Newell, Williams and
//     Dunlop (1993), a weighted second difference (weights 2, -1, -1 per
//     axis) of f (diagonal) and g (off-diagonal) over the corner lattice;
//   far: N_ij = -(V/4 pi) <(3 w_i w_j - |w|^2 delta_ij)/|w|^5>, the dipole
//     tensor averaged over the triangular density of destination-minus-source
//     offsets with Gauss-Legendre quadrature on each half axis; the number of
//     points per half axis falls from 8 to 2 with distance (the paper's
//     "number of integration points chosen by distance"), keeping the
//     relative error near 1e-12 where Newell's cancellation would not.
// The octant is mirrored into the padded grid with the parities of each
// component (xx, yy, zz even; xy odd in x, y; xz odd in x, z; yz odd in y, z;
// every displacement with |i| >= nx is zero), scaled by -mu0/(px py pz),
// Fourier transformed in FP64, and the real spectrum's octant kept in FP32.
#include <math.h>

#include "mm_internal.h"

namespace mm {

// Gauss-Legendre nodes/weights on [-1, 1] for n = 1..8, table offset n(n-1)/2.
constexpr int GL_MAXN = 8;
constexpr int GL_TABLE = GL_MAXN * (GL_MAXN + 1) / 2;

__global__ void k_gauss_legendre(double* nodes, double* weights) {
    const int n = threadIdx.x + 1;  // one thread per order
    if (n > GL_MAXN) return;
    const int off = n * (n - 1) / 2;
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;  // Legendre recurrence
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pn = (n == 1) ? x : p1, pm = (n == 1) ? 1.0 : p0;
            dp = n * (x * pn - pm) / (x * x - 1.0);
            const double dx = pn / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double pn = (n == 1) ? x : p1, pm = (n == 1) ? 1.0 : p0;
        dp = n * (x * pn - pm) / (x * x - 1.0);
        nodes[off + i] = x;
        weights[off + i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

__device__ inline double newell_f(double x, double y, double z) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double r = sqrt(x2 + y2 + z2);
    double o = (2.0 * x2 - y2 - z2) * r / 6.0;
    const double rxz = sqrt(x2 + z2), rxy = sqrt(x2 + y2);
    if (rxz > 0.0) o += 0.5 * y * (z2 - x2) * asinh(y / rxz);
    if (rxy > 0.0) o += 0.5 * z * (y2 - x2) * asinh(z / rxy);
    if (x * r != 0.0) o -= x * y * z * atan(y * z / (x * r));
    return o;
}

__device__ inline double newell_g(double x, double y, double z) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double r = sqrt(x2 + y2 + z2);
    double o = -x * y * r / 3.0;
    const double rxy = sqrt(x2 + y2), ryz = sqrt(y2 + z2), rxz = sqrt(x2 + z2);
    if (rxy > 0.0) o += x * y * z * asinh(z / rxy);
    if (ryz > 0.0) o += y / 6.0 * (3.0 * z2 - y2) * asinh(x / ryz);
    if (rxz > 0.0) o += x / 6.0 * (3.0 * z2 - x2) * asinh(y / rxz);
    if (z * r != 0.0) o -= z2 * z / 6.0 * atan(x * y / (z * r));
    if (y * r != 0.0) o -= z * y2 / 2.0 * atan(x * z / (y * r));
    if (x * r != 0.0) o -= z * x2 / 2.0 * atan(y * z / (x * r));
    return o;
}

// weighted 27-point sum with per-axis weights (2 at 0, -1 at +-1), / (4 pi V)
template <bool DIAG>
__device__ inline double newell_sum(double a, double b, double c, double da, double db, double dc) {
    double s = 0.0;
    for (int p = -1; p <= 1; ++p) {
        const double wp = p == 0 ? 2.0 : -1.0;
        for (int q = -1; q <= 1; ++q) {
            const double wq = q == 0 ? 2.0 : -1.0;
            for (int r = -1; r <= 1; ++r) {
                const double wr = r == 0 ? 2.0 : -1.0;
                const double x = a + p * da, y = b + q * db, z = c + r * dc;
                s += wp * wq * wr * (DIAG ? newell_f(x, y, z) : newell_g(x, y, z));
            }
        }
    }
    return s / (4.0 * M_PI * da * db * dc);
}

__device__ inline int far_order(double rho) {
    if (rho < 4.0) return 8;
    if (rho < 6.0) return 6;
    if (rho < 12.0) return 5;
    if (rho < 50.0) return 4;
    if (rho < 400.0) return 3;
    return 2;
}

__global__ void __launch_bounds__(256) k_tensor_octant(int nx, int ny, int nz, double dx, double dy,
                                                       double dz, const double* __restrict__ gln,
                                                       const double* __restrict__ glw,
                                                       double* __restrict__ out) {
    const long long n = (long long)nx * ny * nz;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int i = (int)(id % nx);
    const long long rest = id / nx;
    const int j = (int)(rest % ny), k = (int)(rest / ny);
    const double X = i * dx, Y = j * dy, Z = k * dz;
    const double diag = sqrt(dx * dx + dy * dy + dz * dz);
    const double rho = sqrt(X * X + Y * Y + Z * Z) / diag;
    double t[6];
    if (rho < 2.5) {
        t[0] = newell_sum<true>(X, Y, Z, dx, dy, dz);
        t[1] = newell_sum<true>(Y, X, Z, dy, dx, dz);
        t[2] = newell_sum<true>(Z, Y, X, dz, dy, dx);
        t[3] = newell_sum<false>(X, Y, Z, dx, dy, dz);
        t[4] = newell_sum<false>(X, Z, Y, dx, dz, dy);
        t[5] = newell_sum<false>(Y, Z, X, dy, dz, dx);
    } else {
        const int ng = far_order(rho);
        const int off = ng * (ng - 1) / 2;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        // nodes on each half axis [0, h] and [-h, 0] with density (h - |s|)/h^2
        for (int a = 0; a < 2 * ng; ++a) {
            const int ia = a % ng;
            const double sa = (a < ng ? 1.0 : -1.0) * 0.5 * dx * (1.0 + gln[off + ia]);
            const double wa = 0.5 * dx * glw[off + ia] * (dx - fabs(sa)) / (dx * dx);
            const double ux = X + sa;
            for (int b = 0; b < 2 * ng; ++b) {
                const int ib = b % ng;
                const double sb = (b < ng ? 1.0 : -1.0) * 0.5 * dy * (1.0 + gln[off + ib]);
                const double wb = 0.5 * dy * glw[off + ib] * (dy - fabs(sb)) / (dy * dy);
                const double uy = Y + sb;
                const double wab = wa * wb;
                for (int c = 0; c < 2 * ng; ++c) {
                    const int ic = c % ng;
                    const double sc = (c < ng ? 1.0 : -1.0) * 0.5 * dz * (1.0 + gln[off + ic]);
                    const double wc = 0.5 * dz * glw[off + ic] * (dz - fabs(sc)) / (dz * dz);
                    const double uz = Z + sc;
                    const double r2 = ux * ux + uy * uy + uz * uz;
                    const double ir = 1.0 / sqrt(r2);
                    const double ir5 = ir * ir * ir * ir * ir;
                    const double w = wab * wc * ir5;
                    acc[0] += w * (3.0 * ux * ux - r2);
                    acc[1] += w * (3.0 * uy * uy - r2);
                    acc[2] += w * (3.0 * uz * uz - r2);
                    acc[3] += w * 3.0 * ux * uy;
                    acc[4] += w * 3.0 * ux * uz;
                    acc[5] += w * 3.0 * uy * uz;
                }
            }
        }
        const double pre = -dx * dy * dz / (4.0 * M_PI);
        for (int c = 0; c < 6; ++c) t[c] = pre * acc[c];
    }
    for (int c = 0; c < 6; ++c) out[c * n + id] = t[c];
}

hipError_t demag_tensor_octant(int nx, int ny, int nz, double dx, double dy, double dz, double* out,
                               hipStream_t s) {
    double* gl = nullptr;
    hipError_t e = hipMalloc((void**)&gl, 2 * GL_TABLE * sizeof(double));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gauss_legendre, dim3(1), dim3(64), 0, s, gl, gl + GL_TABLE);
    const long long n = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_tensor_octant, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nx, ny, nz, dx,
                       dy, dz, gl, gl + GL_TABLE, out);
    e = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(gl);
    return e != hipSuccess ? e : e2;
}

// ---------------------------------------------------------------------------
// Periodic images (paragraph "Periodic boundary conditions"): the kernel entry
// of box displacement (i, j, k) is the sum of N over the displacements
// i + s nx (and likewise along y, z) that stay inside the window |d| <= n P - 1
// of a periodic axis; a non-periodic axis keeps d = i.  The window tensor is
// stored for d >= 0 (lengths wx, wy, wz); a negative d takes the parity of the
// component along that axis.  With these sums in place of the octant, the
// mirror fill below gives the displacement -d the entry of the box
// displacement n - d (the sums satisfy S(n - d) = parity S(d)), so the padded
// linear convolution becomes the cyclic one along the periodic axes.
__global__ void __launch_bounds__(256) k_fold_images(int nx, int ny, int nz, int wx, int wy, int wz, int qx,
                                                     int qy, int qz, const double* __restrict__ win,
                                                     double* __restrict__ oct) {
    const long long n = (long long)nx * ny * nz;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int i = (int)(id % nx);
    const long long rest = id / nx;
    const int j = (int)(rest % ny), k = (int)(rest / ny);
    const long long wn = (long long)wx * wy * wz;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int sz = -qz; sz <= qz; ++sz) {
        const int dk = k + sz * nz;
        if (dk <= -wz || dk >= wz) continue;
        const int ak = dk < 0 ? -dk : dk;
        const bool nzg = dk < 0;
        for (int sy = -qy; sy <= qy; ++sy) {
            const int dj = j + sy * ny;
            if (dj <= -wy || dj >= wy) continue;
            const int aj = dj < 0 ? -dj : dj;
            const bool nyg = dj < 0;
            for (int sx = -qx; sx <= qx; ++sx) {
                const int di = i + sx * nx;
                if (di <= -wx || di >= wx) continue;
                const int ai = di < 0 ? -di : di;
                const bool nxg = di < 0;
                const long long e = ((long long)ak * wy + aj) * wx + ai;
                acc[0] += win[e];
                acc[1] += win[wn + e];
                acc[2] += win[2 * wn + e];
                acc[3] += (nxg != nyg ? -1.0 : 1.0) * win[3 * wn + e];  // xy: odd in x, y
                acc[4] += (nxg != nzg ? -1.0 : 1.0) * win[4 * wn + e];  // xz: odd in x, z
                acc[5] += (nyg != nzg ? -1.0 : 1.0) * win[5 * wn + e];  // yz: odd in y, z
            }
        }
    }
    for (int c = 0; c < 6; ++c) oct[c * n + id] = acc[c];
}

hipError_t demag_fold_images(int nx, int ny, int nz, const int* w, const int* pbc, const double* win,
                             double* oct, hipStream_t s) {
    const long long n = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_fold_images, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nx, ny, nz, w[0], w[1],
                       w[2], pbc[0], pbc[1], pbc[2], win, oct);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mirror fill of component c into the complex FP64 padded array.
__global__ void __launch_bounds__(256) k_mirror_fill(int nx, int ny, int nz, int px, int py, int pz,
                                                     int comp, const double* __restrict__ oct, double scale,
                                                     double2* __restrict__ work) {
    const long long ptot = (long long)px * py * pz;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= ptot) return;
    const int x = (int)(id % px);
    const long long rest = id / px;
    const int y = (int)(rest % py), z = (int)(rest / py);
    // displacement index along each axis; none inside the padding gap
    auto disp = [](int q, int n, int p, int& d, int& sgn) {
        if (q < n) {
            d = q;
            sgn = 1;
            return true;
        }
        if (q > p - n) {
            d = p - q;
            sgn = -1;
            return true;
        }
        return false;
    };
    int di, dj, dk, si, sj, sk;
    double v = 0.0;
    if (disp(x, nx, px, di, si) && disp(y, ny, py, dj, sj) && disp(z, nz, pz, dk, sk)) {
        // parities: comp 0..2 even; 3 = xy odd in x,y; 4 = xz odd in x,z; 5 = yz odd in y,z
        int sign = 1;
        if (comp == 3) sign = si * sj;
        if (comp == 4) sign = si * sk;
        if (comp == 5) sign = sj * sk;
        v = sign * scale * oct[(long long)comp * nx * ny * nz + ((long long)dk * ny + dj) * nx + di];
    }
    work[id] = make_double2(v, 0.0);
}

// One workgroup transforms one line of length p (power of two <= 4096) in
// LDS with radix-2 Stockham stages; twiddles from FP64 sincospi.
__global__ void __launch_bounds__(256) k_fft64_lines(double2* __restrict__ data, int p, int logp,
                                                     long long stride, long long n_inner,
                                                     long long inner_stride, long long outer_stride) {
    extern __shared__ double2 sh64[];
    double2* A = sh64;
    double2* B = sh64 + p;
    const long long l = blockIdx.x;
    const long long off = (l % n_inner) * inner_stride + (l / n_inner) * outer_stride;
    for (int i = threadIdx.x; i < p; i += blockDim.x) A[i] = data[off + i * stride];
    __syncthreads();
    for (int L = 1; L < p; L <<= 1) {
        for (int j = threadIdx.x; j < p / 2; j += blockDim.x) {
            const int k = j & (L - 1);
            const double2 a = A[j], b = A[j + p / 2];
            double s, c;
            sincospi(-(double)k / (double)L, &s, &c);  // exp(-2 pi i k / (2L))
            const double2 bw = make_double2(b.x * c - b.y * s, b.x * s + b.y * c);
            const int o = (j - k) * 2 + k;
            B[o] = make_double2(a.x + bw.x, a.y + bw.y);
            B[o + L] = make_double2(a.x - bw.x, a.y - bw.y);
        }
        __syncthreads();
        double2* t = A;
        A = B;
        B = t;
    }
    for (int i = threadIdx.x; i < p; i += blockDim.x) data[off + i * stride] = A[i];
    (void)logp;
}

// Keep Re of the spectrum's non-negative octant as FP32, in the layout the
// convolution pass reads: [kx][ky_h][kz_h][ncomp] (ncomp = 4 when nz == 1:
// xx, yy, zz, xy; else 6).
__global__ void __launch_bounds__(256) k_extract(int px, int py, int pz, int comp, int ncomp, int kx,
                                                 const double2* __restrict__ work, float* __restrict__ khat) {
    const int kyh = py / 2 + 1, kzh = pz / 2 + 1;
    const long long n = (long long)kx * kyh * kzh;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int ix = (int)(id % kx);
    const long long rest = id / kx;
    const int iy = (int)(rest % kyh), iz = (int)(rest / kyh);
    const double v = work[((long long)iz * py + iy) * px + ix].x;
    const long long dst = (((long long)ix * kyh + iy) * kzh + iz) * ncomp + comp;
    khat[dst] = (float)v;
}

hipError_t demag_kernel_spectrum(int nx, int ny, int nz, int px, int py, int pz, const double* octant,
                                 double2* work, float* khat, int ncomp, int kx, hipStream_t s) {
    const long long ptot = (long long)px * py * pz;
    const double scale = -MU0 / (double)ptot;
    const int nb = (int)((ptot + 255) / 256);
    for (int comp = 0; comp < ncomp; ++comp) {
        hipLaunchKernelGGL(k_mirror_fill, dim3(nb), dim3(256), 0, s, nx, ny, nz, px, py, pz, comp, octant,
                           scale, work);
        const int P[3] = {px, py, pz};
        for (int ax = 0; ax < 3; ++ax) {
            const int p = P[ax];
            if (p == 1) continue;
            long long stride, n_inner, inner_stride, outer_stride, nlines;
            if (ax == 0) {
                stride = 1; nlines = (long long)py * pz; n_inner = nlines; inner_stride = px; outer_stride = 0;
            } else if (ax == 1) {
                stride = px; nlines = (long long)px * pz; n_inner = px; inner_stride = 1;
                outer_stride = (long long)px * py;
            } else {
                stride = (long long)px * py; nlines = (long long)px * py; n_inner = nlines; inner_stride = 1;
                outer_stride = 0;
            }
            const size_t lds = 2 * (size_t)p * sizeof(double2);
            (void)hipFuncSetAttribute((const void*)k_fft64_lines, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
            hipLaunchKernelGGL(k_fft64_lines, dim3((unsigned)nlines), dim3(256), lds, s, work, p, 0, stride,
                               n_inner, inner_stride, outer_stride);
        }
        const long long ne = (long long)kx * (py / 2 + 1) * (pz / 2 + 1);
        hipLaunchKernelGGL(k_extract, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, px, py, pz, comp,
                           ncomp, kx, work, khat);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mm
