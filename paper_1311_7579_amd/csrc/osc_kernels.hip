// HIP kernels of libosc for gfx950 (CDNA4, wave64).
//
// One wave64 owns one tile of kTileEvents consecutive events.  Lane l of
// tile t handles events t*T + m*64 + l, m = 0..K-1 (coalesced SoA loads),
// computes the oscillation probability of each event in FP64 (flavour
// basis, one amplitude element per event), optionally writes it, and adds
// w * P into a lane-private histogram held in LDS.  The 64 lane histograms
// of the tile meet in a fixed binary tree; a merge kernel adds the tile
// results per bin in a fixed binary tree.  No atomics: the bits of the
// histogram do not depend on the launch shape.
#include "osc_internal.h"
#include "osc_launch.h"

namespace osc {

namespace {

constexpr double kSqrt3Half = 0.86602540378443864676;

// Roots of x^3 - tr x^2 + c1 x - det (three real roots: the matrix is
// Hermitian) by the trigonometric solution of the depressed cubic.
__device__ __forceinline__ void cubic_roots(double tr, double c1, double det,
                                            double& l0, double& l1, double& l2)
{
    const double p = fma(tr, tr, -3.0 * c1);                  // tr^2 - 3 c1 >= 0
    const double q = fma(tr, fma(2.0 * tr, tr, -9.0 * c1), 27.0 * det);
    const double sp = sqrt(p);
    double r = q / (2.0 * p * sp);
    r = fmin(1.0, fmax(-1.0, r));
    const double th = acos(r) * (1.0 / 3.0);
    double s, c;
    sincos(th, &s, &c);
    const double k = (2.0 / 3.0) * sp;
    const double t3 = tr * (1.0 / 3.0);
    const double hc = -0.5 * c, hs = kSqrt3Half * s;
    l0 = fma(k, c, t3);
    l1 = fma(k, hc + hs, t3);   // cos(th - 2 pi / 3)
    l2 = fma(k, hc - hs, t3);   // cos(th + 2 pi / 3)
}

// P(alpha -> beta) of one event.  The evolution operator over L is
// sum_k exp(-i phi_k) X_k with the spectral projectors
// X_k = (M - l_j)(M - l_l) / ((l_k - l_j)(l_k - l_l)); the common phase
// exp(-i phi_0) drops out of |.|^2, so only the differences phi_k - phi_0
// are formed.
__device__ __forceinline__ double event_prob(const SetConsts& sc, const Chan* tab,
                                             double kA, double kL, double E, uint32_t f)
{
    const uint32_t a = f & 3u, b = (f >> 2) & 3u;
    const uint32_t idx = (f >> 5) ? 3u : ((b << 2) | a);   // stray high bits -> NaN entry
    const double s = ((f >> 4) & 1u) ? -1.0 : 1.0;
    const Chan c = tab[idx];
    const double A = s * kA * E;
    const double dee = (idx == 0u) ? 1.0 : 0.0;          // alpha = beta = e
    const double dba = (a == b) ? 1.0 : 0.0;

    // amplitude inputs: M_ba and (M^2)_ba (conjugated for antineutrinos)
    const double mre = fma(A, dee, c.m_re);
    const double mim = s * c.m_im;
    const double m2re = fma(A, fma(A, dee, c.g_re), c.m2_re);
    const double m2im = s * fma(A, c.g_im, c.m2_im);

    // matter eigenvalues
    double l0, l1, l2;
    cubic_roots(sc.T0 + A, fma(A, sc.CA, sc.C0), A * sc.DA, l0, l1, l2);

    const double d01 = l0 - l1, d02 = l0 - l2, d12 = l1 - l2;
    const double Q = d01 * d02 * d12;
    const double R = 1.0 / (E * Q);
    const double invE = Q * R, invQ = E * R;
    const double ph = kL * invE;
    double s1, c1, s2, c2;
    sincos(-d01 * ph, &s1, &c1);   // phi_1 - phi_0
    sincos(-d02 * ph, &s2, &c2);   // phi_2 - phi_0
    const double iD0 = d12 * invQ, iD1 = -d02 * invQ, iD2 = d01 * invQ;

    // numerators N_k = (M^2)_ba - (l_j + l_l) M_ba + l_j l_l [a = b]
    const double u0 = l1 + l2, v0 = l1 * l2;
    const double u1 = l0 + l2, v1 = l0 * l2;
    const double u2 = l0 + l1, v2 = l0 * l1;
    const double x0r = fma(v0, dba, fma(-u0, mre, m2re)) * iD0;
    const double x0i = fma(-u0, mim, m2im) * iD0;
    const double x1r = fma(v1, dba, fma(-u1, mre, m2re)) * iD1;
    const double x1i = fma(-u1, mim, m2im) * iD1;
    const double x2r = fma(v2, dba, fma(-u2, mre, m2re)) * iD2;
    const double x2i = fma(-u2, mim, m2im) * iD2;

    // S' = X0 + exp(-i dphi1) X1 + exp(-i dphi2) X2
    const double sr = x0r + c1 * x1r + s1 * x1i + c2 * x2r + s2 * x2i;
    const double si = x0i + c1 * x1i - s1 * x1r + c2 * x2i - s2 * x2r;
    return sr * sr + si * si;
}

__device__ __forceinline__ int bin_of(double x, const BinConsts& bc)
{
    const double q = (x - bc.lo) / bc.wb;
    return (q < 0.0) ? bc.nb : ((q < (double)bc.nb) ? (int)q : bc.nb + 1);
}

// Lane-private histogram slot: bin-major rows of 64 lanes, the lane index
// XOR-swizzled by the bin so that both the per-lane accumulation and the
// per-bin transposed reads spread over the LDS banks.
__device__ __forceinline__ int hslot(int bin, int lane)
{
    return bin * kTileLanes + (lane ^ (bin & 31));
}

// complete binary tree over the 64 lane sums of one bin
template <int N, int J0>
__device__ __forceinline__ double lane_tree(const double* h, int bin)
{
    if constexpr (N == 1) {
        return h[hslot(bin, J0)];
    } else {
        const double left = lane_tree<N / 2, J0>(h, bin);
        const double right = lane_tree<N / 2, J0 + N / 2>(h, bin);
        return left + right;
    }
}

enum Mode { kReweight = 0, kPdf = 1, kHist = 2 };

template <int MODE, bool WRITE_P>
__global__ __launch_bounds__(kTileLanes) void tile_kernel(
    SetConsts sc, PathConsts pc, BinConsts bc, int64_t n, int64_t ntiles,
    const double* __restrict__ e_true, const uint8_t* __restrict__ flags,
    const double* __restrict__ weight, const double* __restrict__ e_reco,
    const double* __restrict__ value, double* __restrict__ p_out,
    double* __restrict__ partial)
{
    extern __shared__ double hist[];
    __shared__ Chan tab[16];

    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kTileEvents + lane;
    const int nbt = bc.nb + 2;

    if (MODE != kHist) {
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 16; ++k) tab[k] = sc.ch[k];
        }
    }
    if (MODE != kReweight) {
        for (int bin = 0; bin < nbt; ++bin) hist[hslot(bin, lane)] = 0.0;
    }
    __syncthreads();

    // all loads of the tile first: K independent coalesced loads per stream
    double ev[kLaneEvents], wv[kLaneEvents], xv[kLaneEvents];
    uint32_t fv[kLaneEvents];
#pragma unroll
    for (int m = 0; m < kLaneEvents; ++m) {
        const int64_t i = base + int64_t(m) * kTileLanes;
        const bool in = i < n;
        if (MODE != kHist) {
            ev[m] = in ? e_true[i] : 1.0;
            fv[m] = in ? flags[i] : 0u;
        } else {
            ev[m] = in ? value[i] : 0.0;
        }
        if (MODE != kReweight) {
            wv[m] = in ? weight[i] : 0.0;
            xv[m] = in ? e_reco[i] : 0.0;
        }
    }

#pragma unroll 2
    for (int m = 0; m < kLaneEvents; ++m) {
        const int64_t i = base + int64_t(m) * kTileLanes;
        if (i < n) {
            double P;
            if (MODE != kHist) {
                P = event_prob(sc, tab, pc.kA, pc.kL, ev[m], fv[m]);
                if (WRITE_P) p_out[i] = P;
            } else {
                P = ev[m];
            }
            if (MODE != kReweight) {
#pragma clang fp contract(off)
                const double cval = wv[m] * P;          // rounded, never fused
                const int slot = hslot(bin_of(xv[m], bc), lane);
                hist[slot] = hist[slot] + cval;          // ascending m per lane
            }
        }
    }

    if (MODE != kReweight) {
        __syncthreads();
        for (int bin = lane; bin < nbt; bin += kTileLanes) {
            partial[int64_t(bin) * ntiles + tile] = lane_tree<kTileLanes, 0>(hist, bin);
        }
    }
}

// In-place complete binary tree over v[0..cnt) (cnt a power of two) by the
// whole block; the result is left in v[0].
__device__ __forceinline__ void block_tree(double* v, int cnt)
{
    for (int s = 1; s < cnt; s <<= 1) {
        __syncthreads();
        for (int p = threadIdx.x; p * 2 * s < cnt; p += blockDim.x) {
            const int i = p * 2 * s;
            v[i] = v[i] + v[i + s];
        }
    }
    __syncthreads();
}

// One block per histogram entry: complete binary tree over the tile
// results padded with +0.0 to a power of two, in chunks of kMergeChunk
// (each chunk is an aligned complete subtree).
__global__ __launch_bounds__(kMergeThreads) void merge_kernel(
    const double* __restrict__ partial, int64_t ntiles, int64_t p2, double* __restrict__ hist_out)
{
    __shared__ double v[kMergeChunk];
    __shared__ double top[kMaxChunks > 0 ? kMaxChunks : 1];
    const int bin = blockIdx.x;
    const int64_t chunk = p2 < kMergeChunk ? p2 : kMergeChunk;
    const int64_t nchunks = p2 / chunk;
    const double* src = partial + int64_t(bin) * ntiles;

    for (int64_t c = 0; c < nchunks; ++c) {
        __syncthreads();
        for (int t = threadIdx.x; t < chunk; t += blockDim.x) {
            const int64_t g = c * chunk + t;
            v[t] = g < ntiles ? src[g] : 0.0;
        }
        block_tree(v, int(chunk));
        if (threadIdx.x == 0) top[c] = v[0];
    }
    block_tree(top, int(nchunks));
    if (threadIdx.x == 0) hist_out[bin] = ntiles > 0 ? top[0] : 0.0;
}

}  // namespace

hipError_t launch_tiles(int mode, bool write_p, const SetConsts& sc, const PathConsts& pc,
                        const BinConsts& bc, int64_t n, const double* e_true,
                        const uint8_t* flags, const double* weight, const double* e_reco,
                        const double* value, double* p_out, double* partial,
                        hipStream_t stream)
{
    const int64_t ntiles = (n + kTileEvents - 1) / kTileEvents;
    if (ntiles == 0) return hipSuccess;
    const size_t lds = mode == kReweight ? 0 : size_t(bc.nb + 2) * kTileLanes * sizeof(double);
    const dim3 grid{unsigned(ntiles)}, block{unsigned(kTileLanes)};
    if (mode == kReweight) {
        hipLaunchKernelGGL((tile_kernel<kReweight, true>), grid, block, lds, stream, sc, pc, bc, n,
                           ntiles, e_true, flags, weight, e_reco, value, p_out, partial);
    } else if (mode == kPdf && write_p) {
        hipLaunchKernelGGL((tile_kernel<kPdf, true>), grid, block, lds, stream, sc, pc, bc, n,
                           ntiles, e_true, flags, weight, e_reco, value, p_out, partial);
    } else if (mode == kPdf) {
        hipLaunchKernelGGL((tile_kernel<kPdf, false>), grid, block, lds, stream, sc, pc, bc, n,
                           ntiles, e_true, flags, weight, e_reco, value, p_out, partial);
    } else {
        hipLaunchKernelGGL((tile_kernel<kHist, false>), grid, block, lds, stream, sc, pc, bc, n,
                           ntiles, e_true, flags, weight, e_reco, value, p_out, partial);
    }
    return hipGetLastError();
}

hipError_t launch_merge(const double* partial, int64_t n, int nbt, double* hist_out,
                        hipStream_t stream)
{
    const int64_t ntiles = (n + kTileEvents - 1) / kTileEvents;
    int64_t p2 = 1;
    while (p2 < ntiles) p2 <<= 1;
    hipLaunchKernelGGL(merge_kernel, dim3(nbt), dim3(kMergeThreads), 0, stream, partial, ntiles,
                       p2, hist_out);
    return hipGetLastError();
}

hipError_t set_kernel_attributes(size_t max_dyn_lds)
{
    const void* fns[] = {
        reinterpret_cast<const void*>(&tile_kernel<kPdf, true>),
        reinterpret_cast<const void*>(&tile_kernel<kPdf, false>),
        reinterpret_cast<const void*>(&tile_kernel<kHist, false>),
    };
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           int(max_dyn_lds));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace osc
