// hswo_levels.hip -- CDNA4 (gfx950) kernels of the HSWO / HSEG / RHSEG hot path:
// leaf initialisation, reassembly of a level from its children, seam
// edges, union-find compression and the per-level label snapshots.

#include "dev_common.h"

namespace hswo {

// ---------------------------------------------------------------------------
// Initialisation, reassembly, compression and snapshots.
// ---------------------------------------------------------------------------
__global__ void k_init_pixels(int32_t* parent, int32_t* mtime, int64_t n) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        parent[p] = (int32_t)p;
        mtime[p] = INT_MAX;
    }
}

// Batch sections: labels are local pixel indices of each section.
__global__ void k_init_pixels_secs(const SecDev* __restrict__ secs) {
    const SecDev& s = secs[blockIdx.y];
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < s.R0; p += gridDim.x * blockDim.x) {
        s.parent[p] = p;
        s.mtime[p] = INT_MAX;
    }
}

template <typename T>
__device__ __forceinline__ float load_px(const void* cube, size_t idx) {
    return (float)reinterpret_cast<const T*>(cube)[idx];
}

template <>
__device__ __forceinline__ float load_px<__half>(const void* cube, size_t idx) {
    return __half2float(reinterpret_cast<const __half*>(cube)[idx]);
}

// Every pixel of a leaf section becomes a region (HSEG step 1): label = its
// pixel index, one pixel, band sums = its spectrum; plus the section's grid
// edges under 4- or 8-connectivity.
template <typename T>
__global__ void k_init_leaves(const SecDev* __restrict__ secs, const InitDev* __restrict__ init,
                              unsigned long long* counters) {
    const SecDev& s = secs[blockIdx.y];
    const InitDev in = init[blockIdx.y];
    const int h = in.h, w = in.w, B = s.B, Bp = s.Bp;
    const int P = h * w;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // band sums and mean rows; non-finite values are counted (the call then stops)
    unsigned nonfinite = 0;
    for (int64_t idx = t0; idx < (int64_t)P * Bp; idx += stride) {
        const int k = (int)(idx / Bp), b = (int)(idx % Bp);
        const int r = k / w, c = k % w;
        float v = 0.0f;
        if (b < B) {
            v = load_px<T>(in.cube, ((size_t)(in.r0 + r) * in.img_w + (in.c0 + c)) * B + b);
            nonfinite += isfinite(v) ? 0u : 1u;
            s.sums[(size_t)k * B + b] = (double)v;
        }
        s.mean[(size_t)k * Bp + b] = v;
    }
    if (nonfinite) atomicAdd(&counters[C_NONFINITE], (unsigned long long)nonfinite);
    // per-pixel region data
    for (int64_t k = t0; k < P; k += stride) {
        const int r = (int)k / w, c = (int)k % w;
        s.label[k] = (in.r0 + r) * in.label_w + (in.c0 + c);
        s.npix[k] = 1;
        s.mark[k] = -1;
        const size_t base = ((size_t)(in.r0 + r) * in.img_w + (in.c0 + c)) * B;
        double nrm = 0.0;
        for (int b = 0; b < B; ++b) {
            const double v = (double)load_px<T>(in.cube, base + b);
            nrm += v * v;
        }
        s.norm[k] = (float)(sqrt(nrm) * (1.0 + 0x1p-20));
    }
    // grid edges in pixel order: pixel k owns slots k*nf .. k*nf+nf-1 for its
    // right, down (and, under 8-connectivity, down-right, down-left)
    // neighbours, so the two rows of consecutive edges stay close. Slots
    // without a neighbour hold (-1,-1): the screen gives them +inf bounds and
    // the first merge's order-preserving compaction removes them.
    const int nf = in.conn == 8 ? 4 : 2;
    const int64_t E0 = (int64_t)P * nf;
    for (int64_t e = t0; e < E0; e += stride) {
        const int k = (int)(e / nf), f = (int)(e % nf);
        const int r = k / w, c = k % w;
        int a = -1, b = -1;
        if (f == 0 && c + 1 < w) {
            a = k;
            b = k + 1;
        } else if (f == 1 && r + 1 < h) {
            a = k;
            b = k + w;
        } else if (f == 2 && r + 1 < h && c + 1 < w) {
            a = k;
            b = k + w + 1;
        } else if (f == 3 && r + 1 < h && c >= 1) {
            a = k;
            b = k + w - 1;
        }
        s.edges[e] = make_int2(a, b);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.st[0] = P;
        s.st[1] = (int)E0;
        s.st[2] = P;
        s.st[3] = 0;
        s.st[4] = 0;
        s.st[5] = 0;
        s.st[6] = 0;
        s.st[7] = 0;
        s.st[8] = 0;
        s.st[9] = 0;
        s.st[10] = 0;
        s.st[11] = 0;
        s.st[12] = 0;
    }
}

// Path compression of the label union-find: parent[p] becomes p's root.
// Concurrent updates only ever store an ancestor, so every walk still ends
// at the root.
__global__ void k_compress(int32_t* parent, int64_t n, const unsigned long long* gate) {
    if (gated(gate)) return;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        int x = parent[p];
        for (int64_t step = 0; step < n; ++step) {  // a chain is never longer than n
            const int y = parent[x];
            if (y == x) break;
            x = y;
        }
        parent[p] = x;
    }
}

__global__ void k_empty() {}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Reassembly (Figure 4.4), part 1: the parent's regions are the live regions
// of its four children in order TL, TR, BL, BR; children's edges are kept.
__global__ void k_assemble(const SecDev* __restrict__ parents, const SecDev* __restrict__ children,
                           const AsmDev* __restrict__ asm_, int32_t* slotmap, const unsigned long long* gate) {
    if (gated(gate)) return;
    const SecDev p = parents[blockIdx.y];
    const AsmDev a = asm_[blockIdx.y];
    int off[5], eoff[5];
    off[0] = 0;
    eoff[0] = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        off[c + 1] = off[c] + children[a.child0 + c].st[0];
        eoff[c + 1] = eoff[c] + children[a.child0 + c].st[1];
    }
    if (off[4] > p.R0 || eoff[4] > p.Ecap) {
        // cannot happen when every child pass ran to its stop count (sections
        // are connected); never write past the parent's capacity
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            p.st[0] = 0;
            p.st[1] = 0;
            p.st[2] = 0;
            p.st[3] = 0;
            p.st[4] = 0;
            p.st[5] = 0;
            p.st[6] = 0;
            p.st[7] = 0;
            p.st[8] = 0;
            p.st[9] = 0;
            p.st[10] = 0;
            p.st[11] = 0;
            p.st[12] = 0;
        }
        return;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int B = p.B, Bp = p.Bp;
    for (int c = 0; c < 4; ++c) {
        const SecDev ch = children[a.child0 + c];
        const int Rc = off[c + 1] - off[c], Ec = eoff[c + 1] - eoff[c];
        for (int64_t k = t0; k < Rc; k += stride) {
            const int ps = off[c] + (int)k;
            const int lab = ch.label[k];
            p.label[ps] = lab;
            p.npix[ps] = ch.npix[k];
            p.norm[ps] = ch.norm[k];
            p.mark[ps] = -1;
            slotmap[lab] = ps;
        }
        for (int64_t idx = t0; idx < (int64_t)Rc * B; idx += stride)
            p.sums[(size_t)off[c] * B + idx] = ch.sums[idx];
        for (int64_t idx = t0; idx < (int64_t)Rc * Bp; idx += stride)
            p.mean[(size_t)off[c] * Bp + idx] = ch.mean[idx];
        for (int64_t e = t0; e < Ec; e += stride) {
            const int2 ed = ch.edges[e];
            // empty slots (a child that made no merge still has them) stay empty
            p.edges[eoff[c] + e] = ed.x < 0 ? make_int2(-1, -1) : make_int2(ed.x + off[c], ed.y + off[c]);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.st[0] = off[4];
        p.st[1] = eoff[4];
        p.st[2] = off[4];
        p.st[3] = 0;
        p.st[4] = 0;
        p.st[5] = 0;
        p.st[6] = 0;
        p.st[7] = 0;
        p.st[8] = 0;
        p.st[9] = 0;
        p.st[10] = 0;
        p.st[11] = 0;
        p.st[12] = 0;
    }
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// Reassembly, part 2: link the regions on either side of the two split lines
// (pixel pairs in different quadrants that are neighbours under the seam
// connectivity), one edge per distinct region pair.
__global__ void k_seam(const SecDev* __restrict__ parents, const AsmDev* __restrict__ asm_,
                       const int32_t* __restrict__ slotmap, const unsigned long long* gate) {
    if (gated(gate)) return;
    const SecDev p = parents[blockIdx.y];
    const AsmDev a = asm_[blockIdx.y];
    const int h0 = a.h / 2, w0 = a.w / 2;
    const int rs = a.r0 + h0 - 1;      // row above the horizontal split
    const int cs0 = a.c0 + w0 - 1;     // columns either side of the vertical split
    const int ncand = a.w + 2 * a.h;   // candidate pixels: that row, those two columns
    const int noff = a.seam_conn == 8 ? 4 : 2;
    const int dr[4] = {0, 1, 1, 1};
    const int dc[4] = {1, 0, 1, -1};
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)ncand * noff;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(idx / noff), o = (int)(idx % noff);
        int r, c;
        if (ci < a.w) {
            r = rs;
            c = a.c0 + ci;
        } else {
            const int k = ci - a.w;
            r = a.r0 + (k >> 1);
            c = cs0 + (k & 1);
        }
        if (r < a.r0 || c < a.c0 || c >= a.c0 + a.w) continue;
        const int r2 = r + dr[o], c2 = c + dc[o];
        if (r2 >= a.r0 + a.h || c2 < a.c0 || c2 >= a.c0 + a.w) continue;
        const int q1 = (r - a.r0 >= h0 ? 2 : 0) + (c - a.c0 >= w0 ? 1 : 0);
        const int q2 = (r2 - a.r0 >= h0 ? 2 : 0) + (c2 - a.c0 >= w0 ? 1 : 0);
        if (q1 == q2) continue;
        const int la = p.parent[(size_t)r * a.img_w + c];
        const int lb = p.parent[(size_t)r2 * a.img_w + c2];
        if (la == lb) continue;
        int sa = slotmap[la], sb = slotmap[lb];
        if (sa > sb) {
            const int t = sa; sa = sb; sb = t;
        }
        const unsigned long long key = ((unsigned long long)(unsigned)sa << 32) | (unsigned)sb;
        unsigned long long hsh = mix64(key) & (unsigned long long)(a.hash_cap - 1);
        for (int probe = 0; probe < a.hash_cap; ++probe) {
            const unsigned long long old = atomicCAS(&a.hash[hsh], ~0ull, key);
            if (old == ~0ull) {
                const int e = atomicAdd(&p.st[1], 1);
                p.edges[e] = make_int2(sa, sb);
                break;
            }
            if (old == key) break;
            hsh = (hsh + 1) & (unsigned long long)(a.hash_cap - 1);
        }
    }
}

// Label maps of the requested hierarchy levels of a top pass. A level with
// count c is the state after k = max(0, R_start - c) top-pass merges: walk
// from the pixel's region at the start of the pass along merges made before k.
__global__ void k_snapshot(const SnapDev* __restrict__ snaps, const int32_t* __restrict__ counts, int n_levels,
                           const unsigned long long* gate) {
    if (gated(gate)) return;
    const SnapDev sd = snaps[blockIdx.y];
    const int P = sd.h * sd.w;
    const int Rs = sd.st[2];
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)P * n_levels;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int lvl = (int)(idx / P), k = (int)(idx % P);
        const int r = k / sd.w, c = k % sd.w;
        const int kcut = Rs - counts[lvl] > 0 ? Rs - counts[lvl] : 0;
        int x = (sd.r0 + r) * sd.label_w + (sd.c0 + c);
        int steps = 0;
        while (sd.mtime[x] < kcut && steps <= P) {  // bounded: a valid chain is shorter than P
            x = sd.parent[x];
            ++steps;
        }
        sd.labels[idx] = steps > P ? -1 : x;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline int grid_for(int64_t n, int bs, int cap) {
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_init_pixels(int32_t* parent, int32_t* mtime, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_init_pixels, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, parent, mtime, n);
    return hipGetLastError();
}

hipError_t launch_init_pixels_secs(const SecDev* secs, int n, int max_pixels, hipStream_t s) {
    hipLaunchKernelGGL(k_init_pixels_secs, dim3(grid_for(max_pixels, 256, 256), n), dim3(256), 0, s, secs);
    return hipGetLastError();
}

hipError_t launch_init_leaves(const SecDev* secs, const InitDev* init, int n, int dtype, int max_pixels,
                              unsigned long long* counters, hipStream_t s) {
    const dim3 grid(grid_for((int64_t)max_pixels * 8, 256, 1024), n);
    if (dtype == HSWO_F16)
        hipLaunchKernelGGL(k_init_leaves<__half>, grid, dim3(256), 0, s, secs, init, counters);
    else
        hipLaunchKernelGGL(k_init_leaves<float>, grid, dim3(256), 0, s, secs, init, counters);
    return hipGetLastError();
}

hipError_t launch_compress(int32_t* parent, int64_t n, const unsigned long long* gate, hipStream_t s) {
    hipLaunchKernelGGL(k_compress, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, parent, n, gate);
    return hipGetLastError();
}

hipError_t launch_empty(hipStream_t s) {
    hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for((int64_t)n, 256, 4096)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_assemble(const SecDev* parents, const SecDev* children, const AsmDev* asm_, int n,
                           int32_t* slotmap, int max_cap, const unsigned long long* gate, hipStream_t s) {
    const dim3 grid(grid_for((int64_t)max_cap * 64, 256, 512), n);
    hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, s, parents, children, asm_, slotmap, gate);
    return hipGetLastError();
}

hipError_t launch_seam(const SecDev* parents, const AsmDev* asm_, int n, const int32_t* slotmap, int max_seam,
                       const unsigned long long* gate, hipStream_t s) {
    const dim3 grid(grid_for((int64_t)max_seam * 4, 256, 256), n);
    hipLaunchKernelGGL(k_seam, grid, dim3(256), 0, s, parents, asm_, slotmap, gate);
    return hipGetLastError();
}

hipError_t launch_snapshot(const SnapDev* snaps, int n, const int32_t* counts, int n_levels, int max_pixels,
                           const unsigned long long* gate, hipStream_t s) {
    const dim3 grid(grid_for((int64_t)max_pixels * n_levels, 256, 4096), n);
    hipLaunchKernelGGL(k_snapshot, grid, dim3(256), 0, s, snaps, counts, n_levels, gate);
    return hipGetLastError();
}

}  // namespace hswo
