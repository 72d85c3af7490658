// Octree of Appendix C on the GPU: bounding cube, Morton codes, a stable LSD
// radix sort of (code, index), level boxes, parents, neighbour and far-field
// lists.  The encoding is fixed so that it can be reproduced bit for bit:
//   lo_d = min_beta s_{beta,d},  ext = max_d (max_beta s_{beta,d} - lo_d),
//   inv = 2^21 / ext,  q_d = min(floor((s_d - lo_d) * inv), 2^21 - 1)
// (one IEEE subtraction then one IEEE multiplication, never fused),
//   code = bit-interleave(q_x, q_y, q_z) (x in bit 3b, y in 3b+1, z in 3b+2),
//   Morton order = stable ascending sort by (code, node index),
//   level-l key = code >> 3(21 - l), parent key = key >> 3,
//   neighbours = same-level boxes with integer coordinates within 1 per axis,
//   FF(l,q) = Children(Neighbor(Parent(l,q))) \ Neighbor(l,q)   (Appendix C).
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "plan.h"

namespace fmb {

namespace {

constexpr int TPB = 256;

__global__ void k_bbox_partial(const double *__restrict__ pts, int64_t n, double *__restrict__ part) {
    __shared__ double sm[6][TPB];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            double v = pts[3 * i + d];
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    }
    for (int d = 0; d < 3; ++d) {
        sm[d][threadIdx.x] = mn[d];
        sm[3 + d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                sm[d][threadIdx.x] = fmin(sm[d][threadIdx.x], sm[d][threadIdx.x + s]);
                sm[3 + d][threadIdx.x] = fmax(sm[3 + d][threadIdx.x], sm[3 + d][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sm[threadIdx.x][0];
}

// params: lo[3], ext, inv
__global__ void k_bbox_final(const double *__restrict__ part, int nb, double *__restrict__ params) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nb; ++b)
        for (int d = 0; d < 3; ++d) {
            mn[d] = fmin(mn[d], part[6 * b + d]);
            mx[d] = fmax(mx[d], part[6 * b + 3 + d]);
        }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) ext = fmax(ext, __dsub_rn(mx[d], mn[d]));
    params[0] = mn[0];
    params[1] = mn[1];
    params[2] = mn[2];
    params[3] = ext;
    params[4] = ext > 0.0 ? __ddiv_rn(2097152.0, ext) : 0.0;   // 2^21 / ext, correctly rounded
}

__device__ inline uint64_t spread3(uint64_t v) {
    // put bit b of v (b < 21) at bit 3b
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

__device__ inline uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ULL;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
    v = (v ^ (v >> 32)) & 0x1fffffULL;
    return (uint32_t)v;
}

__global__ void k_morton(const double *__restrict__ pts, int64_t n, const double *__restrict__ params,
                         uint64_t *__restrict__ codes, int32_t *__restrict__ idx) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv = params[4];
    uint64_t code = 0;
    for (int d = 0; d < 3; ++d) {
        double t = __dmul_rn(__dsub_rn(pts[3 * i + d], params[d]), inv);
        double f = floor(t);
        int64_t q = (int64_t)f;
        if (q > 2097151) q = 2097151;
        if (q < 0) q = 0;
        code |= spread3((uint64_t)q) << d;
    }
    codes[i] = code;
    idx[i] = (int32_t)i;
}

// ---------------- stable LSD radix sort, 4-bit digits ----------------
constexpr int RADIX_ITEMS = 16;
constexpr int RADIX_TILE = TPB * RADIX_ITEMS;

__global__ void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift, int nblocks,
                             int32_t *__restrict__ hist) {
    __shared__ int32_t cnt[16];
    if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RADIX_TILE + (int64_t)threadIdx.x * RADIX_ITEMS;
    int local[16];
    for (int d = 0; d < 16; ++d) local[d] = 0;
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        int64_t i = base + j;
        if (i < n) {
            int d = (int)((keys[i] >> shift) & 15ULL);
#pragma unroll
            for (int q = 0; q < 16; ++q) local[q] += (q == d);
        }
    }
    for (int d = 0; d < 16; ++d)
        if (local[d]) atomicAdd(&cnt[d], local[d]);
    __syncthreads();
    if (threadIdx.x < 16) hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// exclusive scan of a small int array in one block (m up to a few 10^5)
__global__ void k_scan_single(int32_t *__restrict__ a, int64_t m, int32_t *__restrict__ total) {
    __shared__ int32_t sm[TPB];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < m; base += TPB) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < m ? a[i] : 0;
        sm[threadIdx.x] = v;
        __syncthreads();
        for (int s = 1; s < TPB; s <<= 1) {
            int32_t t = threadIdx.x >= s ? sm[threadIdx.x - s] : 0;
            __syncthreads();
            sm[threadIdx.x] += t;
            __syncthreads();
        }
        int32_t incl = sm[threadIdx.x];
        if (i < m) a[i] = carry + incl - v;
        __syncthreads();
        if (threadIdx.x == TPB - 1) carry += incl;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_radix_scatter(const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                uint64_t *__restrict__ kout, int32_t *__restrict__ vout, int64_t n, int shift,
                                int nblocks, const int32_t *__restrict__ hist) {
    __shared__ int32_t pre[16][TPB];
    __shared__ int32_t gbase[16];
    int64_t base = (int64_t)blockIdx.x * RADIX_TILE + (int64_t)threadIdx.x * RADIX_ITEMS;
    int local[16];
    for (int d = 0; d < 16; ++d) local[d] = 0;
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        int64_t i = base + j;
        if (i < n) {
            int d = (int)((kin[i] >> shift) & 15ULL);
#pragma unroll
            for (int q = 0; q < 16; ++q) local[q] += (q == d);
        }
    }
    for (int d = 0; d < 16; ++d) pre[d][threadIdx.x] = local[d];
    if (threadIdx.x < 16) gbase[threadIdx.x] = hist[threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    // exclusive scan of each digit row across threads (Hillis-Steele, in place)
    for (int d = 0; d < 16; ++d) {
        for (int s = 1; s < TPB; s <<= 1) {
            int32_t t = threadIdx.x >= s ? pre[d][threadIdx.x - s] : 0;
            __syncthreads();
            pre[d][threadIdx.x] += t;
            __syncthreads();
        }
    }
    int off[16];
    for (int d = 0; d < 16; ++d) off[d] = gbase[d] + pre[d][threadIdx.x] - local[d];
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        int64_t i = base + j;
        if (i < n) {
            uint64_t k = kin[i];
            int d = (int)((k >> shift) & 15ULL);
            int pos = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (q == d) pos = off[q]++;
            kout[pos] = k;
            vout[pos] = vin[i];
        }
    }
}

// ---------------- device-wide int scans ----------------
__global__ void k_scan_blocks(const int32_t *__restrict__ in, int32_t *__restrict__ out, int64_t m,
                              int32_t *__restrict__ sums) {
    __shared__ int32_t sm[TPB];
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    int32_t v = i < m ? in[i] : 0;
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = 1; s < TPB; s <<= 1) {
        int32_t t = threadIdx.x >= s ? sm[threadIdx.x - s] : 0;
        __syncthreads();
        sm[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < m) out[i] = sm[threadIdx.x];      // inclusive within block
    if (threadIdx.x == TPB - 1) sums[blockIdx.x] = sm[TPB - 1];
}

__global__ void k_scan_add(int32_t *__restrict__ out, int64_t m, const int32_t *__restrict__ sums_excl) {
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < m) out[i] += sums_excl[blockIdx.x];
}

// ---------------- levels ----------------
__global__ void k_level_flags(const uint64_t *__restrict__ codes, int64_t n, int shift, int32_t *__restrict__ flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || (codes[i] >> shift) != (codes[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_level_fill(const uint64_t *__restrict__ codes, int64_t n, int shift, const int32_t *__restrict__ flag,
                             const int32_t *__restrict__ incl, uint64_t *__restrict__ keys, int32_t *__restrict__ start,
                             int32_t *__restrict__ boxid) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t b = incl[i] - 1;
    boxid[i] = b;
    if (flag[i]) {
        keys[b] = codes[i] >> shift;
        start[b] = (int32_t)i;
    }
    if (i == n - 1) start[b + 1] = (int32_t)n;
}

__global__ void k_level_parent(const int32_t *__restrict__ start, int64_t nbox, const int32_t *__restrict__ boxid_prev,
                               int32_t *__restrict__ parent, const uint64_t *__restrict__ keys, int level,
                               const double *__restrict__ params, double *__restrict__ center,
                               int32_t *__restrict__ octant) {
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    parent[b] = level == 0 ? -1 : boxid_prev[start[b]];
    uint64_t key = keys[b];
    octant[b] = (int32_t)(key & 7ULL);
    const double h = params[3] / (double)(1 << level);
    for (int d = 0; d < 3; ++d) {
        uint32_t q = compact3(key >> d);
        center[3 * b + d] = params[d] + ((double)q + 0.5) * h;
    }
}

__global__ void k_child_start(const int32_t *__restrict__ parent_child, int64_t nchild, int64_t nbox_parent,
                              int32_t *__restrict__ child_start) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nchild) return;
    int32_t p = parent_child[c];
    if (c == 0 || parent_child[c - 1] != p) child_start[p] = (int32_t)c;
    if (c == nchild - 1) child_start[nbox_parent] = (int32_t)nchild;
}

__device__ inline int find_key(const uint64_t *__restrict__ keys, int64_t nbox, uint64_t key) {
    int64_t lo = 0, hi = nbox - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        uint64_t v = keys[mid];
        if (v == key) return (int)mid;
        if (v < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

__global__ void k_neighbors(const uint64_t *__restrict__ keys, int64_t nbox, int level, int32_t *__restrict__ nbr) {
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    uint64_t key = keys[b];
    int c[3];
    for (int d = 0; d < 3; ++d) c[d] = (int)compact3(key >> d);
    const int side = 1 << level;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int slot = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                int x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
                int r = -1;
                if (x >= 0 && y >= 0 && z >= 0 && x < side && y < side && z < side) {
                    uint64_t k2 = spread3((uint64_t)x) | (spread3((uint64_t)y) << 1) | (spread3((uint64_t)z) << 2);
                    r = find_key(keys, nbox, k2);
                }
                nbr[b * 27 + slot] = r;
            }
}

// far field: count (ofs == nullptr) or fill
__global__ void k_far_field(const uint64_t *__restrict__ keys, int64_t nbox, const int32_t *__restrict__ parent,
                            const int32_t *__restrict__ nbr_parent, const int32_t *__restrict__ child_start_parent,
                            int32_t *__restrict__ cnt, const int32_t *__restrict__ ofs, int32_t *__restrict__ src,
                            int32_t *__restrict__ op) {
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    int c[3];
    for (int d = 0; d < 3; ++d) c[d] = (int)compact3(keys[b] >> d);
    int32_t p = parent[b];
    int32_t w = ofs ? ofs[b] : 0;
    int32_t count = 0;
    for (int s = 0; s < 27; ++s) {
        int32_t q = nbr_parent[p * 27 + s];
        if (q < 0) continue;
        for (int32_t ch = child_start_parent[q]; ch < child_start_parent[q + 1]; ++ch) {
            int e[3];
            for (int d = 0; d < 3; ++d) e[d] = (int)compact3(keys[ch] >> d) - c[d];
            if (abs(e[0]) <= 1 && abs(e[1]) <= 1 && abs(e[2]) <= 1) continue;
            if (ofs) {
                src[w + count] = ch;
                op[w + count] = (e[0] + 3) * 49 + (e[1] + 3) * 7 + (e[2] + 3);
            }
            ++count;
        }
    }
    if (!ofs) cnt[b] = count;
}

__global__ void k_bucket_count(const int32_t *__restrict__ key, int64_t m, int32_t *__restrict__ cnt) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) atomicAdd(&cnt[key[i]], 1);
}

__global__ void k_bucket_fill(const int32_t *__restrict__ key, int64_t m, int32_t *__restrict__ cursor,
                              int32_t *__restrict__ out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) out[atomicAdd(&cursor[key[i]], 1)] = (int32_t)i;
}

__global__ void k_gather_nodes(const double *__restrict__ pts, const double *__restrict__ nrm,
                               const double *__restrict__ w, const int32_t *__restrict__ tri,
                               const int32_t *__restrict__ perm, int64_t n, double *__restrict__ spts,
                               double *__restrict__ snrm, double *__restrict__ sw, int32_t *__restrict__ stri,
                               int32_t *__restrict__ iperm) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t u = perm[i];
    iperm[u] = (int32_t)i;
    for (int d = 0; d < 3; ++d) {
        spts[3 * i + d] = pts[3 * (int64_t)u + d];
        snrm[3 * i + d] = nrm[3 * (int64_t)u + d];
    }
    sw[i] = w[u];
    stri[i] = tri[u];
}

__global__ void k_p2p_pairs(const int32_t *__restrict__ start, const int32_t *__restrict__ nbr, int64_t nbox,
                            unsigned long long *__restrict__ total) {
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    int64_t ns = 0;
    for (int s = 0; s < 27; ++s) {
        int q = nbr[b * 27 + s];
        if (q >= 0) ns += start[q + 1] - start[q];
    }
    atomicAdd(total, (unsigned long long)(ns * (start[b + 1] - start[b])));
}

__global__ void k_incl_to_excl(int32_t *__restrict__ d, const int32_t *__restrict__ incl, int64_t m) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) d[i] = incl[i] - d[i];
}

inline unsigned grid_for(int64_t m, int tpb = TPB) { return (unsigned)((m + tpb - 1) / tpb); }

// exclusive scan of a device int array (in place), returns the total
int64_t device_exclusive_scan(int32_t *d, int64_t m, hipStream_t s) {
    if (m <= 0) return 0;
    int64_t nb = (m + TPB - 1) / TPB;
    DevBuf incl, sums;
    incl.alloc(m * sizeof(int32_t));
    sums.alloc((nb + 1) * sizeof(int32_t));
    k_scan_blocks<<<nb, TPB, 0, s>>>(d, incl.as<int32_t>(), m, sums.as<int32_t>());
    FMB_LAUNCH_CHECK();
    DevBuf tot;
    tot.alloc(sizeof(int32_t));
    k_scan_single<<<1, TPB, 0, s>>>(sums.as<int32_t>(), nb, tot.as<int32_t>());
    k_scan_add<<<nb, TPB, 0, s>>>(incl.as<int32_t>(), m, sums.as<int32_t>());
    FMB_LAUNCH_CHECK();
    int32_t total = 0;
    FMB_CHECK_HIP(hipMemcpyAsync(&total, tot.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    k_incl_to_excl<<<nb, TPB, 0, s>>>(d, incl.as<int32_t>(), m);
    FMB_LAUNCH_CHECK();
    FMB_CHECK_HIP(hipStreamSynchronize(s));
    return total;
}

}  // namespace

// Number of node pairs that share a triangle but lie in leaves of level d that
// are not neighbours (box coordinates differing by more than one on an axis).
// The near field excludes same-triangle pairs; a pair that the octree hands to
// the far field instead would be counted, so such depths are refused.  code:
// Morton codes in user order; tri: the triangle of each node.
static int64_t split_triangle_pairs(const std::vector<uint64_t> &code, const int32_t *tri, int64_t n, int64_t ntri,
                                    int d) {
    std::vector<int64_t> start(ntri + 1, 0), idx(n);
    for (int64_t i = 0; i < n; ++i) ++start[tri[i] + 1];
    for (int64_t t = 0; t < ntri; ++t) start[t + 1] += start[t];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < n; ++i) idx[fill[tri[i]]++] = i;
    auto coord = [&](uint64_t c, int axis) {
        const uint64_t key = c >> (3 * (NBITS - d));
        int64_t v = 0;
        for (int b = 0; b < d; ++b) v |= (int64_t)((key >> (3 * b + axis)) & 1u) << b;
        return v;
    };
    int64_t bad = 0;
    for (int64_t t = 0; t < ntri; ++t)
        for (int64_t x = start[t]; x < start[t + 1]; ++x)
            for (int64_t y = x + 1; y < start[t + 1]; ++y)
                for (int axis = 0; axis < 3; ++axis)
                    if (std::llabs(coord(code[idx[x]], axis) - coord(code[idx[y]], axis)) > 1) {
                        ++bad;
                        break;
                    }
    return bad;
}

void build_tree(Plan &P, const double *d_pts, hipStream_t s, const int32_t *host_tri) {
    const int64_t n = P.n;
    // bounding cube
    const int nbp = (int)std::min<int64_t>(1024, grid_for(n));
    DevBuf part, params;
    part.alloc(nbp * 6 * sizeof(double));
    params.alloc(8 * sizeof(double));
    k_bbox_partial<<<nbp, TPB, 0, s>>>(d_pts, n, part.as<double>());
    k_bbox_final<<<1, 64, 0, s>>>(part.as<double>(), nbp, params.as<double>());
    FMB_LAUNCH_CHECK();
    double hp[8];
    FMB_CHECK_HIP(hipMemcpyAsync(hp, params.p, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
    FMB_CHECK_HIP(hipStreamSynchronize(s));
    FMB_REQUIRE(hp[3] > 0.0, "all nodes coincide: the bounding cube has zero size");
    P.lo[0] = hp[0];
    P.lo[1] = hp[1];
    P.lo[2] = hp[2];
    P.ext = hp[3];

    // Morton codes and the stable sort by (code, index)
    P.codes.alloc(n * sizeof(uint64_t));
    DevBuf k0, k1, v0, v1;
    k0.alloc(n * sizeof(uint64_t));
    k1.alloc(n * sizeof(uint64_t));
    v0.alloc(n * sizeof(int32_t));
    v1.alloc(n * sizeof(int32_t));
    k_morton<<<grid_for(n), TPB, 0, s>>>(d_pts, n, params.as<double>(), k0.as<uint64_t>(), v0.as<int32_t>());
    FMB_LAUNCH_CHECK();
    FMB_CHECK_HIP(hipMemcpyAsync(P.codes.p, k0.p, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    const int nblk = (int)((n + RADIX_TILE - 1) / RADIX_TILE);
    DevBuf hist;
    hist.alloc((size_t)16 * nblk * sizeof(int32_t));
    uint64_t *kin = k0.as<uint64_t>(), *kout = k1.as<uint64_t>();
    int32_t *vin = v0.as<int32_t>(), *vout = v1.as<int32_t>();
    for (int shift = 0; shift < 64; shift += 4) {
        k_radix_hist<<<nblk, TPB, 0, s>>>(kin, n, shift, nblk, hist.as<int32_t>());
        k_scan_single<<<1, TPB, 0, s>>>(hist.as<int32_t>(), (int64_t)16 * nblk, nullptr);
        k_radix_scatter<<<nblk, TPB, 0, s>>>(kin, vin, kout, vout, n, shift, nblk, hist.as<int32_t>());
        FMB_LAUNCH_CHECK();
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    // 16 passes: the sorted data is back in k0/v0
    const uint64_t *scodes = kin;
    P.perm.alloc(n * sizeof(int32_t));
    FMB_CHECK_HIP(hipMemcpyAsync(P.perm.p, vin, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));

    // level counts for every depth up to MAX_DEPTH (to choose the depth when asked)
    DevBuf flag, incl, sums, boxid_prev, boxid_cur;
    flag.alloc(n * sizeof(int32_t));
    incl.alloc(n * sizeof(int32_t));
    boxid_prev.alloc(n * sizeof(int32_t));
    boxid_cur.alloc(n * sizeof(int32_t));
    const int64_t nb = (n + TPB - 1) / TPB;
    sums.alloc((nb + 1) * sizeof(int32_t));
    auto level_count = [&](int l) -> int64_t {
        const int shift = 3 * (NBITS - l);
        k_level_flags<<<grid_for(n), TPB, 0, s>>>(scodes, n, shift, flag.as<int32_t>());
        k_scan_blocks<<<nb, TPB, 0, s>>>(flag.as<int32_t>(), incl.as<int32_t>(), n, sums.as<int32_t>());
        k_scan_single<<<1, TPB, 0, s>>>(sums.as<int32_t>(), nb, nullptr);
        k_scan_add<<<nb, TPB, 0, s>>>(incl.as<int32_t>(), n, sums.as<int32_t>());
        FMB_LAUNCH_CHECK();
        int32_t last = 0;
        FMB_CHECK_HIP(hipMemcpyAsync(&last, incl.as<int32_t>() + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        return last;
    };
    const bool auto_depth = P.depth == 0;
    if (auto_depth) {
        // deepest level whose mean leaf population still reaches the target
        int d = 2;
        for (; d < MAX_DEPTH; ++d) {
            int64_t nl = level_count(d + 1);
            if ((double)n / (double)nl < (double)P.leaf_target) break;
        }
        P.depth = d;
    }
    if (host_tri && P.ntri > 0 && n > P.ntri) {
        std::vector<uint64_t> hc(n);
        FMB_CHECK_HIP(hipMemcpyAsync(hc.data(), P.codes.p, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        int64_t bad = split_triangle_pairs(hc, host_tri, n, P.ntri, P.depth);
        while (auto_depth && bad > 0 && P.depth > 2) {
            --P.depth;
            bad = split_triangle_pairs(hc, host_tri, n, P.ntri, P.depth);
        }
        FMB_REQUIRE(bad == 0, "the octree is too deep for this mesh: " + std::to_string(bad) +
                                  " node pairs of one triangle fall in leaves that are not neighbours at depth " +
                                  std::to_string(P.depth) + " (their interaction would leave the near field); " +
                                  "use a smaller depth");
    }
    const int L = P.depth;
    P.lv.clear();
    P.lv.resize(L + 1);
    for (int l = 0; l <= L; ++l) {
        Level &V = P.lv[l];
        const int shift = 3 * (NBITS - l);
        V.nbox = level_count(l);
        V.keys.alloc(V.nbox * sizeof(uint64_t));
        V.start.alloc((V.nbox + 1) * sizeof(int32_t));
        V.parent.alloc(V.nbox * sizeof(int32_t));
        V.center.alloc(V.nbox * 3 * sizeof(double));
        V.octant.alloc(V.nbox * sizeof(int32_t));
        V.nbr.alloc(V.nbox * 27 * sizeof(int32_t));
        k_level_fill<<<grid_for(n), TPB, 0, s>>>(scodes, n, shift, flag.as<int32_t>(), incl.as<int32_t>(),
                                                  V.keys.as<uint64_t>(), V.start.as<int32_t>(), boxid_cur.as<int32_t>());
        k_level_parent<<<grid_for(V.nbox), TPB, 0, s>>>(V.start.as<int32_t>(), V.nbox, boxid_prev.as<int32_t>(),
                                                         V.parent.as<int32_t>(), V.keys.as<uint64_t>(), l,
                                                         params.as<double>(), V.center.as<double>(), V.octant.as<int32_t>());
        k_neighbors<<<grid_for(V.nbox), TPB, 0, s>>>(V.keys.as<uint64_t>(), V.nbox, l, V.nbr.as<int32_t>());
        FMB_LAUNCH_CHECK();
        std::swap(boxid_prev, boxid_cur);
        if (l >= 1) {
            Level &U = P.lv[l - 1];
            U.child_start.alloc((U.nbox + 1) * sizeof(int32_t));
            k_child_start<<<grid_for(V.nbox), TPB, 0, s>>>(V.parent.as<int32_t>(), V.nbox, U.nbox,
                                                            U.child_start.as<int32_t>());
            FMB_LAUNCH_CHECK();
        }
    }
    // far-field lists and their grouping by translation vector
    for (int l = 2; l <= L; ++l) {
        Level &V = P.lv[l];
        Level &U = P.lv[l - 1];
        V.ff_ofs.alloc((V.nbox + 1) * sizeof(int32_t));
        FMB_CHECK_HIP(hipMemsetAsync(V.ff_ofs.p, 0, (V.nbox + 1) * sizeof(int32_t), s));
        k_far_field<<<grid_for(V.nbox), TPB, 0, s>>>(V.keys.as<uint64_t>(), V.nbox, V.parent.as<int32_t>(),
                                                      U.nbr.as<int32_t>(), U.child_start.as<int32_t>(),
                                                      V.ff_ofs.as<int32_t>(), nullptr, nullptr, nullptr);
        FMB_LAUNCH_CHECK();
        V.nff = device_exclusive_scan(V.ff_ofs.as<int32_t>(), V.nbox + 1, s);
        V.ff_src.alloc(V.nff * sizeof(int32_t));
        V.ff_op.alloc(V.nff * sizeof(int32_t));
        V.ff_by_op.alloc(V.nff * sizeof(int32_t));
        k_far_field<<<grid_for(V.nbox), TPB, 0, s>>>(V.keys.as<uint64_t>(), V.nbox, V.parent.as<int32_t>(),
                                                      U.nbr.as<int32_t>(), U.child_start.as<int32_t>(), nullptr,
                                                      V.ff_ofs.as<int32_t>(), V.ff_src.as<int32_t>(), V.ff_op.as<int32_t>());
        FMB_LAUNCH_CHECK();
        DevBuf cnt;
        cnt.alloc(N_M2L_OPS * sizeof(int32_t));
        FMB_CHECK_HIP(hipMemsetAsync(cnt.p, 0, N_M2L_OPS * sizeof(int32_t), s));
        if (V.nff > 0) {
            k_bucket_count<<<grid_for(V.nff), TPB, 0, s>>>(V.ff_op.as<int32_t>(), V.nff, cnt.as<int32_t>());
            FMB_LAUNCH_CHECK();
        }
        std::vector<int32_t> hc(N_M2L_OPS);
        FMB_CHECK_HIP(hipMemcpyAsync(hc.data(), cnt.p, N_M2L_OPS * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        V.op_start.assign(N_M2L_OPS + 1, 0);
        for (int o = 0; o < N_M2L_OPS; ++o) V.op_start[o + 1] = V.op_start[o] + hc[o];
        FMB_CHECK_HIP(hipMemcpyAsync(cnt.p, V.op_start.data(), N_M2L_OPS * sizeof(int32_t), hipMemcpyHostToDevice, s));
        if (V.nff > 0) {
            k_bucket_fill<<<grid_for(V.nff), TPB, 0, s>>>(V.ff_op.as<int32_t>(), V.nff, cnt.as<int32_t>(),
                                                           V.ff_by_op.as<int32_t>());
            FMB_LAUNCH_CHECK();
        }
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    }
    // boxes grouped by octant (levels >= 3 feed M2M into level-1; levels >= 3 receive L2L)
    for (int l = 1; l <= L; ++l) {
        Level &V = P.lv[l];
        DevBuf cnt;
        cnt.alloc(8 * sizeof(int32_t));
        FMB_CHECK_HIP(hipMemsetAsync(cnt.p, 0, 8 * sizeof(int32_t), s));
        k_bucket_count<<<grid_for(V.nbox), TPB, 0, s>>>(V.octant.as<int32_t>(), V.nbox, cnt.as<int32_t>());
        FMB_LAUNCH_CHECK();
        int32_t hc[8];
        FMB_CHECK_HIP(hipMemcpyAsync(hc, cnt.p, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        V.oct_start[0] = 0;
        for (int o = 0; o < 8; ++o) V.oct_start[o + 1] = V.oct_start[o] + hc[o];
        FMB_CHECK_HIP(hipMemcpyAsync(cnt.p, V.oct_start.data(), 8 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        V.by_octant.alloc(V.nbox * sizeof(int32_t));
        k_bucket_fill<<<grid_for(V.nbox), TPB, 0, s>>>(V.octant.as<int32_t>(), V.nbox, cnt.as<int32_t>(),
                                                        V.by_octant.as<int32_t>());
        FMB_LAUNCH_CHECK();
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    }
    // near-pair count (statistics)
    {
        DevBuf tot;
        tot.alloc(sizeof(unsigned long long));
        FMB_CHECK_HIP(hipMemsetAsync(tot.p, 0, sizeof(unsigned long long), s));
        k_p2p_pairs<<<grid_for(P.lv[L].nbox), TPB, 0, s>>>(P.lv[L].start.as<int32_t>(), P.lv[L].nbr.as<int32_t>(),
                                                            P.lv[L].nbox, tot.as<unsigned long long>());
        FMB_LAUNCH_CHECK();
        unsigned long long h = 0;
        FMB_CHECK_HIP(hipMemcpyAsync(&h, tot.p, sizeof(h), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        P.p2p_pairs = (int64_t)h;
    }
}

void gather_nodes(Plan &P, const double *d_pts, const double *d_nrm, const double *d_w, const int32_t *d_tri,
                  hipStream_t s) {
    const int64_t n = P.n;
    P.iperm.alloc(n * sizeof(int32_t));
    P.spts.alloc(n * 3 * sizeof(double));
    P.snrm.alloc(n * 3 * sizeof(double));
    P.sw.alloc(n * sizeof(double));
    P.stri.alloc(n * sizeof(int32_t));
    k_gather_nodes<<<grid_for(n), TPB, 0, s>>>(d_pts, d_nrm, d_w, d_tri, P.perm.as<int32_t>(), n, P.spts.as<double>(),
                                                P.snrm.as<double>(), P.sw.as<double>(), P.stri.as<int32_t>(),
                                                P.iperm.as<int32_t>());
    FMB_LAUNCH_CHECK();
    // coincident nodes are refused on the host before the plan is built (a full sort of the coordinates)
}

}  // namespace fmb
