// gc_corr.hpp -- correlation kernels of eqs. (14)-(15) (Sec. 5).
//
// Images are float32, nch channels fastest, given as a window of `rows` x
// `cols` pixels whose rows lie `pitch` pixels apart (pitch = cols for a whole
// image).  All sums are formed in FP64.
//
// Zero shift: one pass of per-channel moments (sum f, sum g, sum f^2,
// sum g^2, sum f g) of the values shifted by the window's first pixel (which
// keeps the centred sums free of cancellation), block partials folded by one
// block; out = { C0, ncc, sum f'^2, sum g'^2, means of f (kCCMaxCh), means
// of g (kCCMaxCh) }.
//
// Every shift (the map of eq. (15)): block (dy, chunk of rows) keeps the
// mean-subtracted FP64 rows j of f and j + dy of g in LDS (the g row padded
// with rx zeros on each side, so that every lane runs the same loop) and
// each lane accumulates sum_i sum_c f'(j, i, c) g'(j + dy, i + dx, c) for its
// shift dx over a segment of the columns; segments are folded through LDS in
// a fixed order, row chunks by a second kernel, also in a fixed order.
#pragma once
#include <hip/hip_runtime.h>

namespace gc {

constexpr int kCCMaxCh = 4;
constexpr int kCCBlocks = 1024;
constexpr int kCCOut = 4 + 2 * kCCMaxCh;      // doubles written by k_cc_final
constexpr int kCCMapMaxDx = 1024;             // 2 rx + 1 at most
constexpr int kCCMapLds = 65536;              // bytes of LDS for the two rows

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// linear pixel index of window pixel p
__device__ __forceinline__ long long win_index(long long p, long long cols, long long pitch)
{
    return cols == pitch ? p : (p / cols) * pitch + p % cols;
}

__global__ void __launch_bounds__(256) k_cc_moments(const float* __restrict__ g, const float* __restrict__ f,
                                                    long long npix, long long cols, long long pitch, int nch,
                                                    double* __restrict__ part)
{
    double m[5][kCCMaxCh];
    double f0[kCCMaxCh], g0[kCCMaxCh];
#pragma unroll
    for (int c = 0; c < kCCMaxCh; ++c) {
        f0[c] = c < nch ? (double)f[c] : 0.0;
        g0[c] = c < nch ? (double)g[c] : 0.0;
#pragma unroll
        for (int q = 0; q < 5; ++q) m[q][c] = 0.0;
    }
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        const long long ix = win_index(p, cols, pitch) * nch;
#pragma unroll
        for (int c = 0; c < kCCMaxCh; ++c) {
            if (c < nch) {
                double a = (double)f[ix + c] - f0[c], b = (double)g[ix + c] - g0[c];
                m[0][c] += a;
                m[1][c] += b;
                m[2][c] += a * a;
                m[3][c] += b * b;
                m[4][c] += a * b;
            }
        }
    }
    __shared__ double red[4][5 * kCCMaxCh];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int c = 0; c < kCCMaxCh; ++c) {
            double v = wave_sum_d(m[q][c]);
            if (lane == 0) red[wave][q * kCCMaxCh + c] = v;
        }
    __syncthreads();
    if (threadIdx.x < 5 * kCCMaxCh) {
        double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        part[(long long)blockIdx.x * 5 * kCCMaxCh + threadIdx.x] = v;
    }
}

// One block of 256: each thread folds the partials of blocks t, t + 256, ...
// for all 5 x kCCMaxCh moments (one pass over the partials), then wave and
// LDS sums.
__global__ void __launch_bounds__(256) k_cc_final(const double* __restrict__ part, int nblocks, long long npix,
                                                  int nch, const float* __restrict__ g, const float* __restrict__ f,
                                                  double* __restrict__ out)
{
    constexpr int Q = 5 * kCCMaxCh;
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const double* pb = part + (long long)b * Q;
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] += pb[q];
    }
    __shared__ double red[4][Q];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double s = wave_sum_d(v[q]);
        if (lane == 0) red[wave][q] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[Q];
        for (int q = 0; q < Q; ++q) tot[q] = red[0][q] + red[1][q] + red[2][q] + red[3][q];
        double sfg = 0.0, sff = 0.0, sgg = 0.0;
        const double N = (double)npix;
        for (int c = 0; c < kCCMaxCh; ++c) {
            out[4 + c] = 0.0;
            out[4 + kCCMaxCh + c] = 0.0;
        }
        for (int c = 0; c < nch; ++c) {
            const double mf = tot[0 * kCCMaxCh + c] / N, mg = tot[1 * kCCMaxCh + c] / N;
            sff += tot[2 * kCCMaxCh + c] - N * mf * mf;
            sgg += tot[3 * kCCMaxCh + c] - N * mg * mg;
            sfg += tot[4 * kCCMaxCh + c] - N * mf * mg;
            out[4 + c] = (double)f[c] + mf;
            out[4 + kCCMaxCh + c] = (double)g[c] + mg;
        }
        out[0] = sfg / sff;
        out[1] = sfg / sqrt(sff * sgg);
        out[2] = sff;
        out[3] = sgg;
    }
}

// Correlation map, partial sums.  Grid (2 ry + 1, n_chunks), 256 threads,
// dynamic LDS of (cols + (cols + 2 rx)) nch doubles.  Task q of thread t is
// t + 256 q: shift index dxi = task % ndx, column segment seg = task / ndx,
// nseg = max(1, 256 / ndx) segments (ndx <= 256: one task per thread;
// otherwise up to 4 shifts per thread over all columns).
__global__ void __launch_bounds__(256) k_cc_map_rows(const float* __restrict__ g, const float* __restrict__ f,
                                                     int rows, int cols, long long pitch, int nch, int rx, int ry,
                                                     int rows_per_chunk, const double* __restrict__ stats,
                                                     double* __restrict__ part)
{
    extern __shared__ double lds[];
    const int ndx = 2 * rx + 1;
    const int nseg = ndx <= 256 ? 256 / ndx : 1;
    const int ntask = ndx * nseg;
    const int n_chunks = gridDim.y;
    const int dy = (int)blockIdx.x - ry;
    const int chunk = blockIdx.y;
    const int t = threadIdx.x;
    double* fs = lds;                            // cols x nch
    double* gs = lds + (long long)cols * nch;    // (cols + 2 rx) x nch, column i at (i + rx)
    const int gw = (cols + 2 * rx) * nch;
    double mf[kCCMaxCh], mg[kCCMaxCh];
#pragma unroll
    for (int c = 0; c < kCCMaxCh; ++c) {
        mf[c] = stats[4 + c];
        mg[c] = stats[4 + kCCMaxCh + c];
    }
    // rows j of f with j + dy inside the window, this chunk's share
    const int jlo = max(0, -dy), jhi = min(rows, rows - dy);
    const int j0 = max(jlo, chunk * rows_per_chunk), j1 = min(jhi, (chunk + 1) * rows_per_chunk);
    // zero padding of the g row (never overwritten below)
    for (int q = t; q < rx * nch; q += blockDim.x) {
        gs[q] = 0.0;
        gs[(cols + rx) * nch + q] = 0.0;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int seg_lo[4], seg_hi[4], dxs[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int task = t + 256 * q;
        const int dxi = task % ndx, seg = task / ndx;
        const bool on = task < ntask;
        dxs[q] = on ? dxi : 0;
        seg_lo[q] = on ? (int)((long long)cols * seg / nseg) : 0;
        seg_hi[q] = on ? (int)((long long)cols * (seg + 1) / nseg) : 0;
    }
    for (int j = j0; j < j1; ++j) {
        __syncthreads();   // the previous row's readers are done
        const float* fr = f + (long long)j * pitch * nch;
        const float* gr = g + (long long)(j + dy) * pitch * nch;
        for (int q = t; q < cols * nch; q += blockDim.x) {
            const int c = q % nch;
            fs[q] = (double)fr[q] - mf[c];
            gs[rx * nch + q] = (double)gr[q] - mg[c];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (seg_hi[q] > seg_lo[q]) {
                // g column i + dx sits at i + dx + rx = i + dxi
                const double* gq = gs + (long long)dxs[q] * nch;
                double s = 0.0;
                for (int e = seg_lo[q] * nch; e < seg_hi[q] * nch; ++e) s += fs[e] * gq[e];
                acc[q] += s;
            }
        }
    }
    (void)gw;
    // fold the column segments of each shift (fixed order), write the chunk's
    // partial sums: part[(dy index * n_chunks + chunk) * ndx + dxi]
    double* out = part + ((long long)blockIdx.x * n_chunks + chunk) * ndx;
    if (nseg > 1) {
        __syncthreads();
        double* red = lds;   // 256 doubles, the rows are no longer needed
        red[t] = acc[0];
        __syncthreads();
        if (t < ndx) {
            double s = 0.0;
            for (int sg = 0; sg < nseg; ++sg) s += red[sg * ndx + t];
            out[t] = s;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int task = t + 256 * q;
            if (task < ntask) out[task] = acc[q];
        }
    }
}

// map[e] = (sum over chunks of part) / sum f'^2, one thread per entry.
__global__ void __launch_bounds__(256) k_cc_map_final(const double* __restrict__ part, int ndx, int ndy,
                                                      int n_chunks, const double* __restrict__ stats,
                                                      double* __restrict__ map)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ndx * ndy) return;
    const int iy = e / ndx, ix = e % ndx;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += part[((long long)iy * n_chunks + c) * ndx + ix];
    map[e] = s / stats[2];
}

// Peak of the map: the maximum and the first (row-major) entry holding it.
// One block of 256; out = { value, dx, dy }.
__global__ void __launch_bounds__(256) k_cc_map_peak(const double* __restrict__ map, int ndx, int ndy, int rx,
                                                     int ry, double* __restrict__ out)
{
    const int n = ndx * ndy;
    double best = -__builtin_huge_val();
    int bi = 0x7fffffff;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const double v = map[e];
        if (v > best) { best = v; bi = e; }   // e rises: the first maximum of this thread's entries
    }
    __shared__ double sv[256];
    __shared__ int si[256];
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double v2 = sv[threadIdx.x + w];
            const int i2 = si[threadIdx.x + w];
            if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int e = si[0];
        out[0] = sv[0];
        out[1] = (double)(e % ndx - rx);
        out[2] = (double)(e / ndx - ry);
    }
}

}  // namespace gc
