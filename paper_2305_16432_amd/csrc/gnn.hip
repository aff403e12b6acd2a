// Preconditioner GNN, forward (Method "Architecture"; technical-details
// appendix): encoders, n_mp message-passing layers, decoder, and the
// lower-triangular assembly L_ij = sqrt(s) (d_ij + d_ji)/2, L_ii =
// sqrt(s) max(softplus(d_ii), 1e-6).
//
// Kernels (H = latent width, 32 or 64; one wave = 32 rows, BF16 MFMA with
// FP32 accumulation, see kern_gnn.h):
//   k_gnn_norm_* per system: s = mean(diag A), rms(b) (two-stage sums)
//   k_enc<NODE>  node encoder on b_i/rms, edge encoder on A_ij/s
//   k_node       aggregation m_i = sum_{k in row i} E[k] * V[col k] (fused),
//                node MLP on [V_i, m_i], and the projections V W_a, V W_b of
//                the edge MLP's first layer (factored: [e, v_i, v_j] W =
//                e W_e + (V W_a)[i] + (V W_b)[j])
//   k_edge<LAST> edge MLP per directed edge; the last layer also runs the
//                decoder and writes the scalar d per edge
//   k_assemble   pair average, softplus diagonal, sqrt(s) scaling
//   k_xdec       optional node decoder on the final node latents: the
//                initial-guess head x^_i (in the frame of A/s and b/rms(b))
#include <algorithm>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "device_util.h"
#include "kern_gnn.h"
#include "lpcg_internal.h"

namespace lpcg {

GnnOff gnn_offsets(int h, int n_mp, bool x_head) {
    GnnOff o{};
    int p = 0;
    auto mlp = [&](MlpOff &m, int fin, int fout) {
        m.W0 = p;
        p += fin * h;
        m.b0 = p;
        p += h;
        m.W1 = p;
        p += h * fout;
        m.b1 = p;
        p += fout;
    };
    mlp(o.node_enc, 1, h);
    mlp(o.edge_enc, 1, h);
    for (int t = 0; t < n_mp; ++t) {
        mlp(o.node[t], 2 * h, h);
        mlp(o.edge[t], 3 * h, h);
    }
    mlp(o.dec, h, 1);
    if (x_head) mlp(o.xdec, h, 1);
    o.total = p;
    return o;
}

// Workspace layout (byte offsets, 256-byte aligned).  Inference keeps two
// V/E buffers (ping-pong); training keeps every layer's activations plus the
// backward pass's intermediates.  The normalisation scalars and the head's
// buffers come first, at offsets common to both layouts.
struct GnnWs {
    size_t sys_s, sys_rms, norm_part;
    size_t V[kMaxMp + 1], Pa[kMaxMp], Pb[kMaxMp], E[kMaxMp + 1], M, Ahat, wpack;
    size_t d, xhat, gxhat;
    // backward (train only)
    size_t gd, gE[2], gV[2], gVmlp, gm, GH, G1, GVN, GH1, H1, Mt, gPa, gPb, HD, GHD, Henc, GHenc, Xn, Xe;
    size_t wpart;
    size_t total;
};

// Layers the fused inference pass supports (its edge chain is unrolled).
constexpr int kFusedMaxMp = 4;

// Packed weights of the fused inference pass (latent width 32): every
// weight the pass kernels keep in LDS, converted once per forward to BF16 in
// MFMA operand order (the LDS image stage_weights writes), 1024 values per
// 32 x 32 image.  Layer u occupies slots (7u .. 7u + 6): 0-1 the node MLP's
// first weight (2H x H, natural order), 2 its second (phi), 3 and 4 the
// node rows W_a, W_b of the edge MLP's first weight (phi), 5 its edge rows
// W_e (phi), 6 the edge MLP's second weight (phi).  After the layers: the
// edge encoder's second weight (natural), the decoder's first (phi), the
// identity (phi) and the node encoder's second weight (natural).
constexpr int kImg = 1024;
__host__ __device__ constexpr int pk_layer(int u, int slot) { return (7 * u + slot) * kImg; }
__host__ __device__ constexpr int pk_glob(int n_mp, int k) { return (7 * n_mp + k) * kImg; }
constexpr int kPkGlob = 4;  // images after the layers
constexpr int kPkEncE = 0, kPkDec = 1, kPkId = 2, kPkEncN = 3;
size_t pack_bytes(int n_mp) { return 2 * (size_t)pk_glob(n_mp, kPkGlob); }

// Blocks of the weight-gradient kernels = number of per-block partial sums.
constexpr int kWgradBlocks = 256;

// Row segments per system for the two-stage normalisation sums: enough for
// the largest system of the batch.
constexpr int kNormRows = 4096;
int norm_segments(const lpcg_system *s) {
    int mx = 1;
    for (int i = 0; i < s->nsys; ++i) mx = std::max(mx, s->h_sys_rowptr[i + 1] - s->h_sys_rowptr[i]);
    return (mx + kNormRows - 1) / kNormRows;
}

// The fused inference pass (k_fused_edge): latent width 32, at most
// kFusedMaxMp layers, and row-aligned edge tiles (no row above 32 entries).
bool gnn_fused(const lpcg_system *s, int h, int n_mp, bool train) {
    return !train && h == 32 && n_mp <= kFusedMaxMp && s->gtiles > 0;
}

GnnWs gnn_ws_layout(const lpcg_system *s, int h, int n_mp, bool train) {
    GnnWs w{};
    const bool fused = gnn_fused(s, h, n_mp, train);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t n = s->n, nnz = s->nnz, mx = std::max(n, nnz);
    w.sys_s = take(sizeof(double) * s->nsys);
    w.sys_rms = take(sizeof(double) * s->nsys);
    w.norm_part = take(2 * sizeof(double) * (size_t)s->nsys * norm_segments(s));
    // the head's output and loss gradient sit before every buffer whose size
    // depends on `train`, at the same offset in both layouts
    w.xhat = take(4 * n);
    w.gxhat = take(4 * n);
    const int nv = train ? n_mp + 1 : 2;
    const int np = train || fused ? n_mp : 1;
    for (int i = 0; i < nv; ++i) w.V[i] = take(2 * n * h);
    for (int i = 0; i < np; ++i) {
        w.Pa[i] = take(2 * n * h);
        w.Pb[i] = take(2 * n * h);
    }
    if (fused) {
        w.M = take(2 * n * h);  // aggregated messages, BF16
        w.wpack = take(pack_bytes(n_mp));
        w.Ahat = take(4 * nnz);  // edge inputs A_e / s, FP32
    }
    else
        for (int i = 0; i < nv; ++i) w.E[i] = take(2 * nnz * h);
    w.d = take(4 * nnz);
    if (train) {
        w.gd = take(4 * nnz);
        w.gE[0] = take(4 * nnz * h);
        w.gE[1] = take(4 * nnz * h);
        w.gV[0] = take(4 * n * h);
        w.gV[1] = take(4 * n * h);
        w.gVmlp = take(4 * n * h);
        w.gm = take(4 * n * h);
        w.GH = take(4 * nnz * h);
        w.G1 = take(2 * nnz * h);
        w.GVN = take(4 * n * h);
        w.GH1 = take(4 * n * h);
        w.H1 = take(2 * n * h);
        w.Mt = take(2 * n * h);
        w.gPa = take(4 * n * h);
        w.gPb = take(4 * n * h);
        w.HD = take(2 * nnz * h);
        w.GHD = take(4 * nnz * h);
        w.Henc = take(2 * mx * h);
        w.GHenc = take(4 * mx * h);
        w.Xn = take(4 * n);
        w.Xe = take(4 * nnz);
        const GnnOff o = gnn_offsets(h, n_mp, true);  // room for the head's weights
        w.wpart = take(sizeof(float) * (size_t)o.total * kWgradBlocks);
    }
    w.total = off;
    return w;
}

namespace {

constexpr int kGnnThreads = 256;  // 4 waves, 32 rows each per tile step
constexpr int kMaxGnnBlocks = 1024;

int nblk(long n, int t) { return (int)((n + t - 1) / t); }

// Copy N BF16 values (N a multiple of 8) from global memory into LDS, 16
// bytes per load; every load of the thread is issued before its first store.
template <int N>
__device__ __forceinline__ void lds_copy(__bf16 *lds, const __bf16 *__restrict__ src) {
    constexpr int C = N / 8, PER = (C + kGnnThreads - 1) / kGnnThreads;
    bf16x8 t[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int g = p * kGnnThreads + threadIdx.x;
        if (g < C) t[p] = *reinterpret_cast<const bf16x8 *>(src + 8 * g);
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int g = p * kGnnThreads + threadIdx.x;
        if (g < C) *reinterpret_cast<bf16x8 *>(lds + 8 * g) = t[p];
    }
}

// One 1024-value unit of the packed weights: values base .. base + 1023 of
// the operand image of a [K x 32] FP32 weight at P + src (row stride ldw;
// phi or natural K order), written from wpack + dst; src < 0: the identity.
struct PackUnit {
    int dst, src, ldw, K, phi, base;
};
struct PackPlan {
    PackUnit u[7 * kFusedMaxMp + kPkGlob];
};

// Unit `unit` of the plan, four values per thread (of 256), loads first.
__device__ __forceinline__ void pack_unit(const float *__restrict__ P, const PackPlan &plan, int unit,
                                          __bf16 *__restrict__ wpack) {
    const PackUnit pu = plan.u[unit];
    const int S = pu.K / 16;
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = pu.base + r * 256 + threadIdx.x;
        const int j = i & 7, lane = (i >> 3) & 63, ms = i >> 9;
        const int st = ms % S, mt = ms / S;
        if (pu.src < 0) v[r] = k_phi(st, j, lane) == (lane & 31) ? 1.f : 0.f;
        else {
            const int k = pu.phi ? k_phi(st, j, lane) : k_nat(st, j, lane);
            v[r] = P[pu.src + (size_t)k * pu.ldw + mt * 32 + (lane & 31)];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) wpack[pu.dst + pu.base + r * 256 + threadIdx.x] = (__bf16)v[r];
}

// Block b writes unit b of the plan.
__global__ void __launch_bounds__(256) k_pack_weights(const float *__restrict__ P, PackPlan plan,
                                                      __bf16 *__restrict__ wpack) {
    pack_unit(P, plan, blockIdx.x, wpack);
}

// Units of the packed weights for n_mp layers (latent width 32).
int pack_plan(const GnnOff &o, int n_mp, PackPlan &plan) {
    constexpr int H = 32;
    int nu = 0;
    auto img = [&](int dst, int src, int ldw, int K, bool phi) {
        for (int base = 0; base < K * H; base += kImg) plan.u[nu++] = PackUnit{dst, src, ldw, K, phi ? 1 : 0, base};
    };
    for (int u = 0; u < n_mp; ++u) {
        img(pk_layer(u, 0), o.node[u].W0, H, 2 * H, false);
        img(pk_layer(u, 2), o.node[u].W1, H, H, true);
        img(pk_layer(u, 3), o.edge[u].W0 + H * H, H, H, true);
        img(pk_layer(u, 4), o.edge[u].W0 + 2 * H * H, H, H, true);
        img(pk_layer(u, 5), o.edge[u].W0, H, H, true);
        img(pk_layer(u, 6), o.edge[u].W1, H, H, true);
    }
    img(pk_glob(n_mp, kPkEncE), o.edge_enc.W1, H, H, false);
    img(pk_glob(n_mp, kPkDec), o.dec.W0, H, H, true);
    img(pk_glob(n_mp, kPkId), -1, 0, H, true);
    img(pk_glob(n_mp, kPkEncN), o.node_enc.W1, H, H, false);
    return nu;
}

// Normalisation sums, stage 1: segment sg (kNormRows rows) of system sy sums
// diag(A) and b^2; empty segments write zeros.
__device__ __forceinline__ void norm_part(int nseg, int sy, int sg, const int *__restrict__ sys_rowptr,
                                          const int *__restrict__ dpos, const double *__restrict__ val,
                                          const double *__restrict__ b, double *__restrict__ part) {
    __shared__ double lds[kGnnThreads / kWave];
    const int r0 = sys_rowptr[sy] + sg * kNormRows;
    const int r1 = min(sys_rowptr[sy + 1], r0 + kNormRows);
    // the thread's rows r0 + threadIdx.x + u * kGnnThreads, summed in that
    // order; all their loads are issued before the first sum
    constexpr int PER = kNormRows / kGnnThreads;
    int ip[PER];
    double bv[PER], dv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = r0 + threadIdx.x + u * kGnnThreads;
        ip[u] = i < r1 ? dpos[i] : -1;
        bv[u] = i < r1 ? b[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) dv[u] = ip[u] >= 0 ? val[ip[u]] : 0.0;
    double sd = 0, sb = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        sd += dv[u];
        sb += bv[u] * bv[u];
    }
    sd = block_sum<kGnnThreads>(sd, lds);
    sb = block_sum<kGnnThreads>(sb, lds);
    if (threadIdx.x == 0) {
        part[2 * ((size_t)sy * nseg + sg)] = sd;
        part[2 * ((size_t)sy * nseg + sg) + 1] = sb;
    }
}

// Block (x, y): segment x of system y.
__global__ void k_gnn_norm_part(int nseg, const int *__restrict__ sys_rowptr, const int *__restrict__ dpos,
                                const double *__restrict__ val, const double *__restrict__ b,
                                double *__restrict__ part) {
    norm_part(nseg, blockIdx.y, blockIdx.x, sys_rowptr, dpos, val, b, part);
}

// The fused inference pass's first launch: blocks (x, y < nsys) the
// normalisation sums, blocks (x < nu, nsys) the weight packing (the two are
// independent, and one launch saves one launch latency).
__global__ void __launch_bounds__(kGnnThreads) k_norm_pack(int nsys, int nseg, const int *__restrict__ sys_rowptr,
                                                           const int *__restrict__ dpos,
                                                           const double *__restrict__ val,
                                                           const double *__restrict__ b, double *__restrict__ part,
                                                           const float *__restrict__ P, PackPlan plan, int nu,
                                                           __bf16 *__restrict__ wpack) {
    if ((int)blockIdx.y < nsys) {
        if ((int)blockIdx.x < nseg) norm_part(nseg, blockIdx.y, blockIdx.x, sys_rowptr, dpos, val, b, part);
    } else if ((int)blockIdx.x < nu) {
        pack_unit(P, plan, blockIdx.x, wpack);
    }
}

// Stage 2: per system, s = mean(diag A) and rms(b) (1 if b = 0), summing the
// segments in order (deterministic).
__global__ void k_gnn_norm_fin(int nsys, int nseg, const int *__restrict__ sys_rowptr,
                               const double *__restrict__ part, double *__restrict__ sys_s,
                               double *__restrict__ sys_rms) {
    const int sy = blockIdx.x * blockDim.x + threadIdx.x;
    if (sy >= nsys) return;
    double sd = 0, sb = 0;
    for (int g = 0; g < nseg; ++g) {
        sd += part[2 * ((size_t)sy * nseg + g)];
        sb += part[2 * ((size_t)sy * nseg + g) + 1];
    }
    const double cnt = (double)(sys_rowptr[sy + 1] - sys_rowptr[sy]);
    sys_s[sy] = sd / cnt;
    const double rms = sqrt(sb / cnt);
    sys_rms[sy] = rms > 0 ? rms : 1.0;
}

// Normalisation finished inside the node encoder (a single system): the
// stage-1 partials of its nseg segments over cnt rows; block 0 stores s and
// rms for the later launches.  part = nullptr: the scale comes from sys_scale.
struct NormIn {
    const double *part;
    int nseg, cnt;
    double *s_out, *rms_out;
};

// Encoder: out[row] = relu(x W0 + b0) W1 + b1 with scalar input x.
template <int H, bool NODE>
__global__ void __launch_bounds__(kGnnThreads) k_enc(int rows, const float *__restrict__ P, MlpOff m,
                                                     const double *__restrict__ xin,
                                                     const int *__restrict__ erow,
                                                     const int *__restrict__ row_sys,
                                                     const double *__restrict__ sys_scale,
                                                     __bf16 *__restrict__ out, float *__restrict__ xs_out,
                                                     const __bf16 *__restrict__ w1p, NormIn nin = NormIn{}) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __align__(16) __bf16 w1[H * H];
    __shared__ double nlds[kGnnThreads / kWave];
    if (w1p) lds_copy<H * H>(w1, w1p);  // packed (the fused inference pass)
    else stage_weights<false>(w1, P + m.W1, H, H, H);
    double own_scale = 1.0;
    if (nin.part) {  // every block alike: s = mean(diag A), rms(b) (1 if b = 0)
        double sd = 0.0, sb = 0.0;
        for (int g = threadIdx.x; g < nin.nseg; g += kGnnThreads) {
            sd += nin.part[2 * g];
            sb += nin.part[2 * g + 1];
        }
        sd = block_sum<kGnnThreads>(sd, nlds);
        sb = block_sum<kGnnThreads>(sb, nlds);
        const double rms = sqrt(sb / nin.cnt);
        own_scale = rms > 0 ? rms : 1.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            nin.s_out[0] = sd / nin.cnt;
            nin.rms_out[0] = own_scale;
        }
    }
    __syncthreads();
    const int lane = lane_id();
    const float *W0 = P + m.W0, *b0 = P + m.b0, *b1 = P + m.b1;
    const int ntiles = (rows + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int r = tile * 32 + (lane & 31);
        const bool valid = r < rows;
        float x = 0.f;
        if (valid) {
            const int node = NODE ? r : erow[r];
            x = (float)(xin[r] / (nin.part ? own_scale : sys_scale[row_sys[node]]));
        }
        f32x16 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            bf16x8 b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = k_nat(s, j, lane);
                b[j] = (__bf16)fmaxf(x * W0[k] + b0[k], 0.f);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma(lds_op(w1, S, mt, s, lane), b, acc[mt]);
        }
        add_bias<MT>(acc, b1, lane, false);
        if (valid) store_acc_bf16<MT>(out + (size_t)r * H, acc, lane);
        if (valid && xs_out && lane < 32) xs_out[r] = x;
    }
}

// Node layer t: V' = f_v([V, m]) with m_i = sum_k E[k] * V[col k]; Pa = V' W_a,
// Pb = V' W_b (rows H..2H-1 and 2H..3H-1 of the edge MLP's first weight).
template <int H>
__global__ void __launch_bounds__(kGnnThreads) k_node(int n, const int *__restrict__ rowptr,
                                                      const int *__restrict__ col,
                                                      const float *__restrict__ P, MlpOff mv, MlpOff me,
                                                      const __bf16 *__restrict__ V,
                                                      const __bf16 *__restrict__ E,
                                                      __bf16 *__restrict__ Vn, __bf16 *__restrict__ Pa,
                                                      __bf16 *__restrict__ Pb) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __bf16 w0[2 * H * H], w1[H * H], wa[H * H], wb[H * H];
    stage_weights<false>(w0, P + mv.W0, H, 2 * H, H);
    stage_weights<true>(w1, P + mv.W1, H, H, H);
    stage_weights<true>(wa, P + me.W0 + H * H, H, H, H);
    stage_weights<true>(wb, P + me.W0 + 2 * H * H, H, H, H);
    __syncthreads();
    const int lane = lane_id();
    const int ntiles = (n + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int i = tile * 32 + (lane & 31);
        const bool valid = i < n;
        bf16x8 bx[2 * S];
        // V part
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (valid) {
                bx[s] = load8(V + (size_t)i * H + k_nat(s, 0, lane));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) bx[s][j] = (__bf16)0.f;
            }
        }
        // aggregated messages m_i (FP32 sums of BF16 products)
        float msum[S][8];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) msum[s][j] = 0.f;
        if (valid) {
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int c = col[k];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const bf16x8 e8 = load8(E + (size_t)k * H + k_nat(s, 0, lane));
                    const bf16x8 v8 = load8(V + (size_t)c * H + k_nat(s, 0, lane));
#pragma unroll
                    for (int j = 0; j < 8; ++j) msum[s][j] += (float)e8[j] * (float)v8[j];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) bx[S + s][j] = (__bf16)msum[s][j];
        // hidden = relu(W0^T [V, m]^T + b0)
        f32x16 hid[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) hid[mt] = zero16();
#pragma unroll
        for (int s = 0; s < 2 * S; ++s)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) hid[mt] = mfma(lds_op(w0, 2 * S, mt, s, lane), bx[s], hid[mt]);
        add_bias<MT>(hid, P + mv.b0, lane, true);
        // V' = W1^T hidden + b1
        f32x16 vo[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) vo[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8 b = acc_operand<MT>(hid, s);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) vo[mt] = mfma(lds_op(w1, S, mt, s, lane), b, vo[mt]);
        }
        add_bias<MT>(vo, P + mv.b1, lane, false);
        if (valid) store_acc_bf16<MT>(Vn + (size_t)i * H, vo, lane);
        // projections of V' for the edge MLP
        f32x16 pa[MT], pb[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            pa[mt] = zero16();
            pb[mt] = zero16();
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8 b = acc_operand<MT>(vo, s);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                pa[mt] = mfma(lds_op(wa, S, mt, s, lane), b, pa[mt]);
                pb[mt] = mfma(lds_op(wb, S, mt, s, lane), b, pb[mt]);
            }
        }
        if (valid) {
            store_acc_bf16<MT>(Pa + (size_t)i * H, pa, lane);
            store_acc_bf16<MT>(Pb + (size_t)i * H, pb, lane);
        }
    }
}

// Edge layer t: E'[e] = f_e([E[e], V'_row, V'_col]) through the factored
// first layer; LAST also runs the decoder d[e] = relu(E' Wd0 + bd0) wd1 + bd1.
template <int H, bool LAST>
__global__ void __launch_bounds__(kGnnThreads) k_edge(int nnz, const int *__restrict__ erow,
                                                      const int *__restrict__ col,
                                                      const float *__restrict__ P, MlpOff me, MlpOff md,
                                                      const __bf16 *__restrict__ E,
                                                      const __bf16 *__restrict__ Pa,
                                                      const __bf16 *__restrict__ Pb,
                                                      __bf16 *__restrict__ En, float *__restrict__ d) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __bf16 we[H * H], w1[H * H], wd[LAST ? H * H : 1];
    stage_weights<false>(we, P + me.W0, H, H, H);
    stage_weights<true>(w1, P + me.W1, H, H, H);
    if (LAST) stage_weights<true>(wd, P + md.W0, H, H, H);
    __syncthreads();
    const int lane = lane_id();
    const int ntiles = (nnz + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int e = tile * 32 + (lane & 31);
        const bool valid = e < nnz;
        const int r = valid ? erow[e] : 0, c = valid ? col[e] : 0;
        f32x16 hid[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) hid[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            bf16x8 b;
            if (valid) {
                b = load8(E + (size_t)e * H + k_nat(s, 0, lane));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = (__bf16)0.f;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) hid[mt] = mfma(lds_op(we, S, mt, s, lane), b, hid[mt]);
        }
        const float *b0 = P + me.b0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = acc_feat(mt, 4 * q, lane);
                bf16x4 ga, gb;
                if (valid) {
                    ga = *reinterpret_cast<const bf16x4 *>(Pa + (size_t)r * H + f);
                    gb = *reinterpret_cast<const bf16x4 *>(Pb + (size_t)c * H + f);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float add = valid ? (float)ga[t] + (float)gb[t] : 0.f;
                    hid[mt][4 * q + t] = fmaxf(hid[mt][4 * q + t] + add + b0[f + t], 0.f);
                }
            }
        f32x16 eo[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) eo[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8 b = acc_operand<MT>(hid, s);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) eo[mt] = mfma(lds_op(w1, S, mt, s, lane), b, eo[mt]);
        }
        add_bias<MT>(eo, P + me.b1, lane, false);
        if (valid && En) store_acc_bf16<MT>(En + (size_t)e * H, eo, lane);
        if (LAST) {
            f32x16 hd[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) hd[mt] = zero16();
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const bf16x8 b = acc_operand<MT>(eo, s);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) hd[mt] = mfma(lds_op(wd, S, mt, s, lane), b, hd[mt]);
            }
            add_bias<MT>(hd, P + md.b0, lane, true);
            const float *w1d = P + md.W1;
            float part = 0.f;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int i = 0; i < 16; ++i) part += hd[mt][i] * w1d[acc_feat(mt, i, lane)];
            part += __shfl_xor(part, 32, kWave);
            if (valid && lane < 32) d[e] = part + P[md.b1];
        }
    }
}

// ---------------------------------------------------------------------------
// Fused inference pass (latent width 32).  The edge latents are never stored:
// E_t[e] is recomputed from the edge input A_e/s through the encoder and the
// chain of edge MLPs 0..t-1, whose node terms (V_u W_a)[row] and
// (V_u W_b)[col] come from the per-layer projections the node passes keep.
// Message-passing pass t computes, per row-aligned tile of at most 32
// entries, the messages E_t[e] * V_t[col e] and their row sums m_i in CSR
// order (through LDS); the node pass then needs only V_t and m.  The last
// pass runs the whole chain and the decoder.  Edge MLP evaluations grow from
// n_mp to n_mp (n_mp + 1) / 2, but no edge latent crosses HBM.  Rounding
// points are those of the stored form: E_t enters each product as BF16, the
// message sum runs in FP32 in CSR order and m enters the node MLP as BF16.
struct FusedChain {
    MlpOff edge[kFusedMaxMp];
    const __bf16 *pa[kFusedMaxMp];
    const __bf16 *pb[kFusedMaxMp];
    const __bf16 *wpack;  // packed weights (pk_layer / pk_glob layout)
    int n_mp;
};

template <int CH, bool DEC>
__global__ void __launch_bounds__(kGnnThreads) k_fused_edge(
    int nnz, int ntiles, const int *__restrict__ tile_row, const int *__restrict__ tile_e,
    const int *__restrict__ rowptr, const int *__restrict__ erow, const int *__restrict__ col,
    const double *__restrict__ aval, const int *__restrict__ row_sys, const double *__restrict__ sys_s,
    float *__restrict__ ahat, const float *__restrict__ P, MlpOff enc, FusedChain ch, MlpOff md,
    const __bf16 *__restrict__ V, __bf16 *__restrict__ M, float *__restrict__ d, int zero) {
    constexpr int H = 32, S = H / 16;
    // FP32 constants: encoder W0, b0, b1; b0, b1 of each chain layer; decoder
    // b0, W1 (a column), b1
    constexpr int C_ENC = 0, C_CH = 3 * H, C_DEC = C_CH + 2 * H * CH, NC = C_DEC + 2 * H + 1;
    // LDS weights, one image each: the encoder's second layer, then W_e and
    // W_1 of each chain layer, the decoder's first layer, the identity
    constexpr int NIMG = 1 + 2 * CH + (DEC ? 1 : 0) + (CH > 0 ? 1 : 0);
    __shared__ __align__(16) __bf16 wl[NIMG][H * H];
    __bf16 *const wenc = wl[0];
    __bf16 *const wd = wl[DEC ? 1 + 2 * CH : 0];
    __bf16 *const wid = wl[CH > 0 ? NIMG - 1 : 0];
    __shared__ __align__(16) float cst[NC];
    __shared__ float msg[DEC ? 1 : kGnnThreads / kWave][DEC ? 1 : 32][H + 1];
    {
        // every 16-byte chunk of the packed images and every constant is
        // loaded before the first LDS store (one memory round trip)
        constexpr int CPI = H * H / 8, CHUNKS = NIMG * CPI;
        constexpr int PER = (CHUNKS + kGnnThreads - 1) / kGnnThreads, PERC = (NC + kGnnThreads - 1) / kGnnThreads;
        const int T = ch.n_mp;
        bf16x8 tv[PER];
        float cv[PERC];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int g = p * kGnnThreads + threadIdx.x;
            if (g < CHUNKS) {
                const int q = g / CPI;
                int off;
                if (q == 0) off = pk_glob(T, kPkEncE);
                else if (q <= 2 * CH) off = pk_layer((q - 1) >> 1, 5 + ((q - 1) & 1));
                else if (DEC && q == 2 * CH + 1) off = pk_glob(T, kPkDec);
                else off = pk_glob(T, kPkId);
                tv[p] = *reinterpret_cast<const bf16x8 *>(ch.wpack + off + 8 * (g % CPI));
            }
        }
#pragma unroll
        for (int p = 0; p < PERC; ++p) {
            const int i = p * kGnnThreads + threadIdx.x;
            float v = 0.f;
            if (i < C_CH) v = P[(i < H ? enc.W0 : i < 2 * H ? enc.b0 - H : enc.b1 - 2 * H) + i];
            else if (i < C_DEC) {
                const int u = (i - C_CH) / (2 * H), k = (i - C_CH) % (2 * H);
                v = k < H ? P[ch.edge[u].b0 + k] : P[ch.edge[u].b1 + k - H];
            } else if (DEC && i < NC) {
                const int k = i - C_DEC;
                v = k < H ? P[md.b0 + k] : k < 2 * H ? P[md.W1 + k - H] : P[md.b1];
            }
            cv[p] = v;
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int g = p * kGnnThreads + threadIdx.x;
            if (g < CHUNKS) *reinterpret_cast<bf16x8 *>(&wl[0][0] + 8 * g) = tv[p];
        }
#pragma unroll
        for (int p = 0; p < PERC; ++p) {
            const int i = p * kGnnThreads + threadIdx.x;
            if (i < NC) cst[i] = cv[p];
        }
    }
    __syncthreads();
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    const int tiles = DEC ? (nnz + 31) / 32 : ntiles;
    const int rr = lane & 31;
    // A tile's index data: its rows and entries, the lane's edge (row r,
    // column c, input x = A_e / s) and the entry range of the row the lane
    // sums.  The next tile's are loaded while the current one computes (one
    // tile ahead, unconditionally: the last tile is re-read at the end), so
    // only the gathers that depend on them wait a full memory round trip.
    struct TileIn {
        int e0, r0, r1, e, r, c, ka, kb;
        bool valid, sums;
        float x;
    };
    auto load_in = [&](int t) {
        TileIn q;
        int e_end;
        if (DEC) {
            q.r0 = q.r1 = q.e0 = 0;
            q.e = t * 32 + rr;
            e_end = nnz;
        } else {
            q.r0 = tile_row[t];
            q.r1 = tile_row[t + 1];
            q.e0 = tile_e[t];
            q.e = q.e0 + rr;
            e_end = tile_e[t + 1];
        }
        q.valid = q.e < e_end;
        const int ec = q.valid ? q.e : 0;
        q.r = erow[ec];
        q.c = col[ec];
        q.sums = !DEC && q.r0 + rr < q.r1;
        const int ra = q.sums ? q.r0 + rr : 0;
        q.ka = rowptr[ra] - q.e0;
        q.kb = rowptr[ra + 1] - q.e0;
        if (CH == 0 && !DEC) q.x = (float)(aval[ec] / sys_s[row_sys[q.r]]);  // first pass: A_e / s
        else q.x = ahat[ec];                                                  // later: as kept
        if (!q.valid) q.x = 0.f;
        return q;
    };
    // XCD-aware mapping: blocks are dispatched round-robin over the 8 XCDs,
    // so block b runs on XCD b % 8; each XCD takes one contiguous eighth of
    // the tiles (rows), and the node rows its tiles gather (the neighbours of
    // a contiguous row range) stay in that XCD's L2.
    const int nx = gridDim.x % 8 == 0 ? 8 : 1;
    const int xcd = blockIdx.x % nx, nbx = gridDim.x / nx;
    const int t_lo = (int)((long)tiles * xcd / nx), t_hi = (int)((long)tiles * (xcd + 1) / nx);
    if (t_lo >= t_hi) return;
    const int stride = nbx * 4;
    int tile = t_lo + (blockIdx.x / nx) * 4 + wv;
    TileIn nxt = load_in(min(tile, t_hi - 1));
    for (; tile < t_hi; tile += stride) {
        const TileIn ti = nxt;
        nxt = load_in(min(tile + stride, t_hi - 1));
        // `zero` is 0 at run time; the compiler cannot prove it, so the weight
        // operands and constants below are re-read from LDS in every tile
        // rather than hoisted into registers for the whole loop (over a
        // hundred registers for a three-layer chain, one wave per SIMD)
        const int z = zero * tile;
        const float *C = cst + z;
        const int e = ti.e, r0 = ti.r0, r = ti.r, c = ti.c, ka = ti.ka, kb = ti.kb;
        const bool valid = ti.valid;
        const float x = ti.x;
        if (CH == 0 && !DEC && valid && lane < 32) ahat[e] = x;  // kept for the later passes
        // every gather of the tile issued up front, so their latencies overlap
        // instead of following each other layer by layer
        bf16x4 gpa[CH > 0 ? CH : 1][4], gpb[CH > 0 ? CH : 1][4], gv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int f = acc_feat(0, 4 * q, lane);
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                gpa[u][q] = *reinterpret_cast<const bf16x4 *>(ch.pa[u] + (size_t)r * H + f);
                gpb[u][q] = *reinterpret_cast<const bf16x4 *>(ch.pb[u] + (size_t)c * H + f);
            }
            if (!DEC) gv[q] = *reinterpret_cast<const bf16x4 *>(V + (size_t)c * H + f);
        }
        // every accumulator starts from its layer's bias (the MFMA adds onto it)
        f32x16 acc[1];
        acc[0] = bias16(C + C_ENC + 2 * H, lane);
#pragma unroll
        for (int st = 0; st < S; ++st) {
            // first encoder layer at this lane's 8 input features k_nat(st, 0..7)
            const int k0 = k_nat(st, 0, lane);
            bf16x8 b;
#pragma unroll
            for (int j4 = 0; j4 < 2; ++j4) {
                const f32x4 w0 = *reinterpret_cast<const f32x4 *>(C + C_ENC + k0 + 4 * j4);
                const f32x4 b0 = *reinterpret_cast<const f32x4 *>(C + C_ENC + H + k0 + 4 * j4);
#pragma unroll
                for (int j = 0; j < 4; ++j) b[4 * j4 + j] = (__bf16)fmaxf(x * w0[j] + b0[j], 0.f);
            }
            acc[0] = mfma(lds_op(wenc + z, S, 0, st, lane), b, acc[0]);
        }
        // edge MLPs 0..CH-1 through the factored first layer: the node terms
        // Pa[row] and Pb[col] enter the accumulator through an identity
        // product, straight from their BF16 gathers (the lane's gathered
        // features are exactly its accumulator features, in phi order)
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            f32x16 hid[1];
            hid[0] = bias16(C + C_CH + 2 * H * u, lane);
#pragma unroll
            for (int st = 0; st < S; ++st) {
                hid[0] = mfma(lds_op(wid + z, S, 0, st, lane), cat8(gpa[u][2 * st], gpa[u][2 * st + 1]), hid[0]);
                hid[0] = mfma(lds_op(wid + z, S, 0, st, lane), cat8(gpb[u][2 * st], gpb[u][2 * st + 1]), hid[0]);
            }
#pragma unroll
            for (int st = 0; st < S; ++st)
                hid[0] = mfma(lds_op(wl[1 + 2 * u] + z, S, 0, st, lane), acc_operand<1>(acc, st), hid[0]);
#pragma unroll
            for (int i = 0; i < 16; ++i) hid[0][i] = relu_bits(hid[0][i]);
            f32x16 out[1];
            out[0] = bias16(C + C_CH + 2 * H * u + H, lane);
#pragma unroll
            for (int st = 0; st < S; ++st)
                out[0] = mfma(lds_op(wl[2 + 2 * u] + z, S, 0, st, lane), acc_operand<1>(hid, st), out[0]);
            acc[0] = out[0];
        }
        if (DEC) {
            // decoder d = relu(E W0 + b0) w1 + b1 (one scalar per edge)
            f32x16 hd[1];
            hd[0] = bias16(C + C_DEC, lane);
#pragma unroll
            for (int st = 0; st < S; ++st) hd[0] = mfma(lds_op(wd + z, S, 0, st, lane), acc_operand<1>(acc, st), hd[0]);
#pragma unroll
            for (int i = 0; i < 16; ++i) hd[0][i] = relu_bits(hd[0][i]);
            float part = 0.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) part += hd[0][i] * C[C_DEC + H + acc_feat(0, i, lane)];
            part += __shfl_xor(part, 32, kWave);
            if (valid && lane < 32) d[e] = part + C[C_DEC + 2 * H];
        } else {
            // messages E_t[e] * V_t[col e] (E_t rounded to BF16 as when stored)
            float(*mw)[H + 1] = msg[wv];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = acc_feat(0, 4 * q, lane);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    mw[lane & 31][f + t] = (float)(__bf16)acc[0][4 * q + t] * (float)gv[q][t];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // row sums in CSR order, one (row, feature) pair per lane and step:
            // pair p = row * H + feature for p = lane, lane + 64, ...; lane rr
            // holds row rr's entry range (ka, kb)
            const int pairs = (ti.r1 - r0) * H;
            for (int pb = 0; pb < pairs; pb += kWave) {
                const int pr = pb + lane;
                const int row = min(pr, pairs - 1) / H, f = pr % H;
                const int a0 = __shfl(ka, row), a1 = __shfl(kb, row);
                float sum = 0.f;
                for (int k = a0; k < a1; ++k) sum += mw[k][f];
                if (pr < pairs) M[(size_t)(r0 + row) * H + f] = (__bf16)sum;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Node layer of the fused pass: V' = f_v([V, m]) with the aggregated
// messages m read from memory; Pa = V' W_a, Pb = V' W_b as in k_node.
template <int H>
__global__ void __launch_bounds__(kGnnThreads) k_node_m(int n, const float *__restrict__ P, MlpOff mv, MlpOff me,
                                                        const __bf16 *__restrict__ V, const __bf16 *__restrict__ M,
                                                        __bf16 *__restrict__ Vn, __bf16 *__restrict__ Pa,
                                                        __bf16 *__restrict__ Pb, const __bf16 *__restrict__ wp) {
    constexpr int S = H / 16, MT = H / 32;
    // the layer's packed images in their packed order: the node MLP's two
    // weights, then W_a and W_b of the edge MLP (one contiguous copy)
    __shared__ __align__(16) __bf16 wl[5 * H * H];
    __bf16 *const w0 = wl, *const w1 = wl + 2 * H * H, *const wa = wl + 3 * H * H, *const wb = wl + 4 * H * H;
    lds_copy<5 * H * H>(wl, wp);
    __syncthreads();
    const int lane = lane_id();
    const int ntiles = (n + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int i = tile * 32 + (lane & 31);
        const bool valid = i < n;
        bf16x8 bx[2 * S];
#pragma unroll
        for (int st = 0; st < S; ++st) {
            if (valid) {
                bx[st] = load8(V + (size_t)i * H + k_nat(st, 0, lane));
                bx[S + st] = load8(M + (size_t)i * H + k_nat(st, 0, lane));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) bx[st][j] = bx[S + st][j] = (__bf16)0.f;
            }
        }
        f32x16 hid[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) hid[mt] = zero16();
#pragma unroll
        for (int st = 0; st < 2 * S; ++st)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) hid[mt] = mfma(lds_op(w0, 2 * S, mt, st, lane), bx[st], hid[mt]);
        add_bias<MT>(hid, P + mv.b0, lane, true);
        f32x16 vo[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) vo[mt] = zero16();
#pragma unroll
        for (int st = 0; st < S; ++st) {
            const bf16x8 b = acc_operand<MT>(hid, st);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) vo[mt] = mfma(lds_op(w1, S, mt, st, lane), b, vo[mt]);
        }
        add_bias<MT>(vo, P + mv.b1, lane, false);
        if (valid) store_acc_bf16<MT>(Vn + (size_t)i * H, vo, lane);
        f32x16 pa[MT], pb[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            pa[mt] = zero16();
            pb[mt] = zero16();
        }
#pragma unroll
        for (int st = 0; st < S; ++st) {
            const bf16x8 b = acc_operand<MT>(vo, st);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                pa[mt] = mfma(lds_op(wa, S, mt, st, lane), b, pa[mt]);
                pb[mt] = mfma(lds_op(wb, S, mt, st, lane), b, pb[mt]);
            }
        }
        if (valid) {
            store_acc_bf16<MT>(Pa + (size_t)i * H, pa, lane);
            store_acc_bf16<MT>(Pb + (size_t)i * H, pb, lane);
        }
    }
}

// softplus(kDiagShift) = 1: the learned diagonal of L' starts at 1 (mode 2).
constexpr float kDiagShift = 0.54132485461291810f;  // ln(e - 1)

__device__ __forceinline__ float softplus_f(float x) { return x > 20.f ? x : log1pf(expf(x)); }

// Mode 3 (diagonal completed): radicand A_ii - sum_{j<i} L_ij^2 of row i, the
// strictly-lower values in the mode-1 form, FP64 sum in row order.  The
// strictly-lower entries of row i are its first (lrowptr[i+1] - lrowptr[i] -
// 1) stored entries of A (columns ascending).
constexpr double kCompleteFloor = 1e-3;
__device__ __forceinline__ double complete_radicand(int i, const int *__restrict__ rowptr,
                                                    const int *__restrict__ lrowptr, const int *__restrict__ col,
                                                    const int *__restrict__ rev, const double *__restrict__ diag64,
                                                    const float *__restrict__ d) {
    const int a = rowptr[i], cnt = lrowptr[i + 1] - lrowptr[i] - 1;
    double ssq = 0.0;
    // four entries at a time, all their loads issued before the first use
    // (past the row's strict entries the loads repeat entry a and the terms
    // are left out); the terms are summed in entry order
    for (int q0 = 0; q0 < cnt; q0 += 4) {
        int c[4], rv[4];
        float dk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = a + (q0 + u < cnt ? q0 + u : 0);
            c[u] = col[k];
            rv[u] = rev[k];
            dk[u] = d[k];
        }
        double dg[4];
        float dr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            dg[u] = diag64[c[u]];
            dr[u] = d[rv[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float l = (float)sqrt(dg[u]) * (0.5f * (dk[u] + dr[u]));
            if (q0 + u < cnt) ssq += (double)l * (double)l;
        }
    }
    return diag64[i] - ssq;
}

// L value of the lower-pattern entry with A-position k.
__device__ __forceinline__ float l_entry(int k, int mode, const int *__restrict__ erow,
                                         const int *__restrict__ col, const int *__restrict__ rev,
                                         const int *__restrict__ row_sys, const double *__restrict__ sys_s,
                                         const double *__restrict__ diag64, const float *__restrict__ d) {
    const int i = erow[k], j = col[k];
    if (mode == 0) {
        const float sq = (float)sqrt(sys_s[row_sys[i]]);
        if (j == i) return sq * fmaxf(softplus_f(d[k]), 1e-6f);
        return sq * 0.5f * (d[k] + d[rev[k]]);
    }
    if (j == i) {
        const float sa = (float)sqrt(diag64[i]);
        return mode == 1 || mode == 3 ? sa : sa * fmaxf(softplus_f(d[k] + kDiagShift), 1e-6f);
    }
    return (float)sqrt(diag64[j]) * (0.5f * (d[k] + d[rev[k]]));
}

// Value of L at L-position q (mode 3 completes the diagonal).
__device__ __forceinline__ float l_value(int q, int mode, const int *__restrict__ lsrc,
                                         const int *__restrict__ rowptr, const int *__restrict__ lrowptr,
                                         const int *__restrict__ erow, const int *__restrict__ col,
                                         const int *__restrict__ rev, const int *__restrict__ row_sys,
                                         const double *__restrict__ sys_s, const double *__restrict__ diag64,
                                         const float *__restrict__ d) {
    const int k = lsrc[q];
    const int i = erow[k];
    if (mode == 3 && col[k] == i) {
        const double rad = complete_radicand(i, rowptr, lrowptr, col, rev, diag64, d);
        const double fl = kCompleteFloor * diag64[i];
        return (float)sqrt(rad > fl ? rad : fl);
    }
    return l_entry(k, mode, erow, col, rev, row_sys, sys_s, diag64, d);
}

// Mode 3 with one thread per row: the row's strictly-lower values and its
// completed diagonal from one set of loads (per entry, each strictly-lower
// value is computed once for its own position and again in its row's
// radicand).  The expressions and the FP64 order of the radicand are those of
// l_value; the row's last L position holds the diagonal.  Entries are taken
// eight at a time, indices clamped into the row, all loads issued before the
// first use.  utval (may be null): each value also goes to its L^T position,
// entry (j, i) of U row j at urowptr[j] + (rev - dpos[j]) (the diagonal first
// in its row), found with the same round of loads as the value's inputs.
__global__ void k_assemble_rows3(int n, const int *__restrict__ lsrc, const int *__restrict__ lrowptr,
                                 const int *__restrict__ col, const int *__restrict__ rev,
                                 const int *__restrict__ urowptr, const int *__restrict__ dpos,
                                 const double *__restrict__ diag64, const float *__restrict__ d,
                                 float *__restrict__ lval, float *__restrict__ utval) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int q0 = lrowptr[i], cnt = lrowptr[i + 1] - q0 - 1;
    const int u0i = urowptr[i];
    const double di = diag64[i];
    double ssq = 0.0;
    for (int u0 = 0; u0 < cnt; u0 += 8) {
        int k[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) k[u] = lsrc[q0 + min(u0 + u, cnt - 1)];
        int c[8], rv[8];
        float dk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c[u] = col[k[u]];
            rv[u] = rev[k[u]];
            dk[u] = d[k[u]];
        }
        double dg[8];
        float dr[8];
        int ur[8], dp[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dg[u] = diag64[c[u]];
            dr[u] = d[rv[u]];
            ur[u] = utval ? urowptr[c[u]] : 0;
            dp[u] = utval ? dpos[c[u]] : 0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (u0 + u < cnt) {
                const float l = (float)sqrt(dg[u]) * (0.5f * (dk[u] + dr[u]));
                lval[q0 + u0 + u] = l;
                if (utval) utval[ur[u] + (rv[u] - dp[u])] = l;
                ssq += (double)l * (double)l;
            }
        }
    }
    const double rad = di - ssq, fl = kCompleteFloor * di;
    const float dv = (float)sqrt(rad > fl ? rad : fl);
    lval[q0 + cnt] = dv;
    if (utval) utval[u0i] = dv;
}

// Transposed copy: ut[p] = l[u2l[p]] (the values k_assemble would compute
// again at those positions).
__global__ void k_gather_ut(int nnz_l, const int *__restrict__ u2l, const float *__restrict__ lval,
                            float *__restrict__ utval) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz_l) utval[p] = lval[u2l[p]];
}

__global__ void k_assemble(int nnz_l, int mode, const int *__restrict__ lsrc, const int *__restrict__ u2l,
                           const int *__restrict__ rowptr, const int *__restrict__ lrowptr,
                           const int *__restrict__ erow, const int *__restrict__ col,
                           const int *__restrict__ rev, const int *__restrict__ row_sys,
                           const double *__restrict__ sys_s, const double *__restrict__ diag64,
                           const float *__restrict__ d, float *__restrict__ lval, float *__restrict__ utval) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz_l) return;
    if (lval) lval[p] = l_value(p, mode, lsrc, rowptr, lrowptr, erow, col, rev, row_sys, sys_s, diag64, d);
    if (utval) utval[p] = l_value(u2l[p], mode, lsrc, rowptr, lrowptr, erow, col, rev, row_sys, sys_s, diag64, d);
}

// Initial-guess head: x^_i = relu(V_i W0 + b0) w1 + b1 on the final node
// latents V = V_T.
template <int H>
__global__ void __launch_bounds__(kGnnThreads) k_xdec(int n, const float *__restrict__ P, MlpOff m,
                                                      const __bf16 *__restrict__ VT, float *__restrict__ xhat) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __bf16 w0[H * H];
    stage_weights<false>(w0, P + m.W0, H, H, H);
    __syncthreads();
    const int lane = lane_id();
    const float *w1 = P + m.W1;
    const int ntiles = (n + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int i = tile * 32 + (lane & 31);
        const bool valid = i < n;
        f32x16 hid[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) hid[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            bf16x8 b;
            if (valid) {
                b = load8(VT + (size_t)i * H + k_nat(s, 0, lane));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = (__bf16)0.f;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) hid[mt] = mfma(lds_op(w0, S, mt, s, lane), b, hid[mt]);
        }
        add_bias<MT>(hid, P + m.b0, lane, true);
        float part = 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int q = 0; q < 16; ++q) part += hid[mt][q] * w1[acc_feat(mt, q, lane)];
        part += __shfl_xor(part, 32, kWave);
        if (valid && lane < 32) xhat[i] = part + P[m.b1];
    }
}

__global__ void k_zero_f32(int n, float *__restrict__ p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

int gnn_blocks(long rows) { return std::max(1, std::min(kMaxGnnBlocks, nblk(rows, 32 * 4))); }

// Grid of a fused-pass kernel: as many 256-thread blocks as the chip holds
// at once (the kernel's occupancy, queried once per kernel, times the
// compute units), never more than one per 4 tiles.  Each wave then loops
// over its tiles, and the whole grid is resident.
int resident_grid(const void *kfn, long tiles) {
    static std::mutex mu;
    static std::vector<std::pair<const void *, int>> cache;
    int per = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (auto &c : cache)
            if (c.first == kfn) per = c.second;
        if (per == 0) {
            int dev = 0, cus = 0, occ = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kfn, kGnnThreads, 0) != hipSuccess || occ <= 0)
                per = kMaxGnnBlocks;
            else
                per = occ * cus;
            cache.emplace_back(kfn, per);
        }
    }
    long g = std::max(1L, std::min((long)per, (tiles + 3) / 4));
    if (g >= 64) g -= g % 8;  // whole XCD rounds (the kernels map tiles per XCD)
    return (int)g;
}

template <int H>
int forward_impl(const lpcg_system *s, const lpcg_gnn *net, const double *b, unsigned char *ws,
                 const GnnWs &L, bool train, float *lval, float *utval, hipStream_t st) {
    const GnnOff o = gnn_offsets(H, net->n_mp, net->x_head != 0);
    const float *P = net->params;
    double *sys_s = (double *)(ws + L.sys_s), *sys_rms = (double *)(ws + L.sys_rms);
    const bool fused = gnn_fused(s, H, net->n_mp, train);  // per-layer projections kept
    const int nseg = norm_segments(s);
    double *npart = (double *)(ws + L.norm_part);
    // the fused pass (width 32) launches the normalisation sums with the
    // weight packing, and a single system's node encoder finishes them
    const bool fused32 = H == 32 && fused;
    const bool enc_norm = fused32 && s->nsys == 1;
    if (!enc_norm) {
        k_gnn_norm_part<<<dim3(nseg, s->nsys), kGnnThreads, 0, st>>>(nseg, s->sys_rowptr, s->dpos, s->val64, b,
                                                                     npart);
        k_gnn_norm_fin<<<nblk(s->nsys, 64), 64, 0, st>>>(s->nsys, nseg, s->sys_rowptr, npart, sys_s, sys_rms);
    }
    auto V = [&](int t) { return (__bf16 *)(ws + L.V[train ? t : (t & 1)]); };
    auto E = [&](int t) { return (__bf16 *)(ws + L.E[train ? t : (t & 1)]); };
    auto Pa = [&](int t) { return (__bf16 *)(ws + L.Pa[train || fused ? t : 0]); };
    auto Pb = [&](int t) { return (__bf16 *)(ws + L.Pb[train || fused ? t : 0]); };
    float *d = (float *)(ws + L.d);
    const int T = net->n_mp;
    if (H == 32 && fused) {
        __bf16 *wpack = (__bf16 *)(ws + L.wpack);
        {
            PackPlan plan{};
            const int nu = pack_plan(o, T, plan);
            if (enc_norm) {
                k_norm_pack<<<dim3(std::max(nseg, nu), 2), kGnnThreads, 0, st>>>(
                    1, nseg, s->sys_rowptr, s->dpos, s->val64, b, npart, P, plan, nu, wpack);
            } else {
                k_pack_weights<<<nu, 256, 0, st>>>(P, plan, wpack);
            }
        }
        const NormIn nin = enc_norm ? NormIn{npart, nseg, s->n, sys_s, sys_rms} : NormIn{};
        k_enc<H, true><<<gnn_blocks(s->n), kGnnThreads, 0, st>>>(s->n, P, o.node_enc, b, s->erow, s->row_sys,
                                                                  sys_rms, V(0), nullptr,
                                                                  wpack + pk_glob(T, kPkEncN), nin);
        __bf16 *M = (__bf16 *)(ws + L.M);
        float *ahat = (float *)(ws + L.Ahat);
        FusedChain ch{};
        ch.wpack = wpack;
        ch.n_mp = T;
        for (int t = 0; t <= T; ++t) {
            const long tiles = t < T ? s->gtiles : (s->nnz + 31) / 32;
            switch (t + (t == T ? 8 : 0)) {
#define LPCG_FUSED(CHN, DECN)                                                                                       \
    k_fused_edge<CHN, DECN><<<resident_grid((const void *)k_fused_edge<CHN, DECN>, tiles), kGnnThreads, 0, st>>>( \
        s->nnz, s->gtiles, s->gtile_row, s->gtile_e, s->rowptr, s->erow, s->colind, s->val64, s->row_sys, sys_s,    \
        ahat, P, o.edge_enc, ch, o.dec, V(t), M, d, 0)
                case 0: LPCG_FUSED(0, false); break;
                case 1: LPCG_FUSED(1, false); break;
                case 2: LPCG_FUSED(2, false); break;
                case 3: LPCG_FUSED(3, false); break;
                case 9: LPCG_FUSED(1, true); break;
                case 10: LPCG_FUSED(2, true); break;
                case 11: LPCG_FUSED(3, true); break;
                default: LPCG_FUSED(4, true); break;
#undef LPCG_FUSED
            }
            if (t == T) break;
            k_node_m<H><<<gnn_blocks(s->n), kGnnThreads, 0, st>>>(s->n, P, o.node[t], o.edge[t], V(t), M, V(t + 1),
                                                                  Pa(t), Pb(t), wpack + pk_layer(t, 0));
            ch.edge[t] = o.edge[t];
            ch.pa[t] = Pa(t);
            ch.pb[t] = Pb(t);
        }
    } else {
    k_enc<H, true><<<gnn_blocks(s->n), kGnnThreads, 0, st>>>(s->n, P, o.node_enc, b, s->erow, s->row_sys,
                                                              sys_rms, V(0),
                                                              train ? (float *)(ws + L.Xn) : nullptr, nullptr);
    k_enc<H, false><<<gnn_blocks(s->nnz), kGnnThreads, 0, st>>>(s->nnz, P, o.edge_enc, s->val64, s->erow,
                                                                 s->row_sys, sys_s, E(0),
                                                                 train ? (float *)(ws + L.Xe) : nullptr, nullptr);
    for (int t = 0; t < T; ++t) {
        k_node<H><<<gnn_blocks(s->n), kGnnThreads, 0, st>>>(s->n, s->rowptr, s->colind, P, o.node[t],
                                                             o.edge[t], V(t), E(t), V(t + 1), Pa(t), Pb(t));
        if (t + 1 < T)
            k_edge<H, false><<<gnn_blocks(s->nnz), kGnnThreads, 0, st>>>(
                s->nnz, s->erow, s->colind, P, o.edge[t], o.dec, E(t), Pa(t), Pb(t), E(t + 1), d);
        else
            k_edge<H, true><<<gnn_blocks(s->nnz), kGnnThreads, 0, st>>>(
                s->nnz, s->erow, s->colind, P, o.edge[t], o.dec, E(t), Pa(t), Pb(t),
                train ? E(t + 1) : nullptr, d);
    }
    }
    // L in its own order, then L^T gathered from it when both are wanted
    // (each value computed once); U alone is assembled directly
    const bool rows3 = net->diag_mode == 3 && lval;
    if (rows3)
        k_assemble_rows3<<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->lsrc, s->lrowptr, s->colind, s->rev,
                                                          s->urowptr, s->dpos, s->diag64, d, lval, utval);
    else
        k_assemble<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, net->diag_mode, s->lsrc, s->u2l, s->rowptr,
                                                         s->lrowptr, s->erow, s->colind, s->rev, s->row_sys,
                                                         sys_s, s->diag64, d, lval, lval ? nullptr : utval);
    if (lval && utval && !rows3) k_gather_ut<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, s->u2l, lval, utval);
    if (net->x_head) {
        k_xdec<H><<<gnn_blocks(s->n), kGnnThreads, 0, st>>>(s->n, P, o.xdec, V(T), (float *)(ws + L.xhat));
        // the head's loss gradient starts at zero: a backward without an
        // initial-guess loss leaves the head's weights with zero gradient
        if (train) k_zero_f32<<<nblk(s->n, 256), 256, 0, st>>>(s->n, (float *)(ws + L.gxhat));
    }
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

int check_net(const lpcg_gnn *net) {
    if (!net || !net->params || (net->h != 32 && net->h != 64) || net->n_mp < 1 || net->n_mp > kMaxMp ||
        net->diag_mode < 0 || net->diag_mode > 3 || net->x_head < 0 || net->x_head > 1) {
        set_error("gnn: h must be 32 or 64, 1 <= n_mp <= %d, diag_mode 0 .. 3, x_head 0 or 1", kMaxMp);
        return LPCG_EINVAL;
    }
    return LPCG_OK;
}

}  // namespace

int gnn_forward(const lpcg_system *s, const lpcg_gnn *net, const double *b, void *ws, int64_t ws_bytes,
                bool train, float *lval, float *utval, hipStream_t st) {
    int rc = check_net(net);
    if (rc) return rc;
    if (!s || !b || !ws) {
        set_error("gnn forward: invalid arguments");
        return LPCG_EINVAL;
    }
    if (s->nsys > 65535) {
        set_error("gnn forward: at most 65535 systems per batch");
        return LPCG_EINVAL;
    }
    const GnnWs L = gnn_ws_layout(s, net->h, net->n_mp, train);
    if ((size_t)ws_bytes < L.total) {
        set_error("gnn forward: workspace of %lld bytes, %zu needed", (long long)ws_bytes, L.total);
        return LPCG_ENOMEM;
    }
    if (s->perm) {  // node inputs in the system's internal order
        if ((rc = to_internal_f64(s, b, s->bperm, st))) return rc;
        b = s->bperm;
    }
    if (net->h == 32) return forward_impl<32>(s, net, b, (unsigned char *)ws, L, train, lval, utval, st);
    return forward_impl<64>(s, net, b, (unsigned char *)ws, L, train, lval, utval, st);
}

}  // namespace lpcg

using namespace lpcg;

extern "C" int64_t lpcg_gnn_param_count(int32_t h, int32_t n_mp, int32_t x_head) {
    if (h <= 0 || n_mp < 1 || n_mp > kMaxMp || x_head < 0 || x_head > 1) return -1;
    return gnn_offsets(h, n_mp, x_head != 0).total;
}

extern "C" int64_t lpcg_gnn_workspace_bytes(const lpcg_system *s, int32_t h, int32_t n_mp, int32_t train) {
    if (!s || h <= 0 || n_mp < 1 || n_mp > kMaxMp) return -1;
    return (int64_t)gnn_ws_layout(s, h, n_mp, train != 0).total;
}

extern "C" int lpcg_gnn_predict_L(const lpcg_system *s, const lpcg_gnn *net, const double *b, void *ws,
                                  int64_t ws_bytes, float *l_val, float *ut_val, hipStream_t st) {
    return gnn_forward(s, net, b, ws, ws_bytes, false, l_val, ut_val, st);
}

extern "C" int lpcg_gnn_forward_train(const lpcg_system *s, const lpcg_gnn *net, const double *b, void *ws,
                                      int64_t ws_bytes, float *l_val, hipStream_t st) {
    return gnn_forward(s, net, b, ws, ws_bytes, true, l_val, nullptr, st);
}

// --------------------------------------------------------------------------
// Initial-guess head (appendix comparing with a predicted starting guess):
// the node decoder regresses the solution of the normalised system
// (A/s) x' = b/rms(b), i.e. x' = x s / rms(b); x0 = x^ rms(b) / s.
namespace lpcg {
namespace {

__global__ void k_x0_scale(int n, const int *__restrict__ row_sys, const double *__restrict__ sys_s,
                           const double *__restrict__ sys_rms, const float *__restrict__ xhat,
                           double *__restrict__ x0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int y = row_sys[i];
    x0[i] = (double)xhat[i] * sys_rms[y] / sys_s[y];
}

// Stage 1 of the head's loss: block (x, y) handles segment x (kNormRows
// rows) of system y: d_i = x^_i - x_i s / rms, gradient w 2 d_i, partial sum
// of d_i^2.
__global__ void k_x0_loss_part(int nseg, const int *__restrict__ sys_rowptr, const double *__restrict__ sys_s,
                               const double *__restrict__ sys_rms, const float *__restrict__ xhat,
                               const double *__restrict__ x, double w, float *__restrict__ gxhat,
                               double *__restrict__ part) {
    __shared__ double lds[kGnnThreads / kWave];
    const int sy = blockIdx.y, sg = blockIdx.x;
    const int r0 = sys_rowptr[sy] + sg * kNormRows;
    const int r1 = min(sys_rowptr[sy + 1], r0 + kNormRows);
    const double scale = sys_s[sy] / sys_rms[sy];
    double acc = 0;
    for (int i = r0 + threadIdx.x; i < r1; i += kGnnThreads) {
        const double d = (double)xhat[i] - x[i] * scale;
        acc += d * d;
        if (gxhat) gxhat[i] = (float)(2.0 * w * d);
    }
    acc = block_sum<kGnnThreads>(acc, lds);
    if (threadIdx.x == 0) part[(size_t)sy * nseg + sg] = acc;
}

__global__ void k_x0_loss_fin(int nsys, int nseg, const double *__restrict__ part, double *__restrict__ loss) {
    const int sy = blockIdx.x * blockDim.x + threadIdx.x;
    if (sy >= nsys) return;
    double acc = 0;
    for (int g = 0; g < nseg; ++g) acc += part[(size_t)sy * nseg + g];
    loss[sy] = acc;
}

int check_head(const lpcg_system *s, const lpcg_gnn *net, const void *ws, int64_t ws_bytes, const char *who) {
    int rc = check_net(net);
    if (rc) return rc;
    if (!s || !ws || !net->x_head) {
        set_error("%s: invalid arguments (the network needs x_head = 1)", who);
        return LPCG_EINVAL;
    }
    const GnnWs L = gnn_ws_layout(s, net->h, net->n_mp, false);
    if ((size_t)ws_bytes < L.total) {
        set_error("%s: workspace of %lld bytes, %zu needed", who, (long long)ws_bytes, L.total);
        return LPCG_ENOMEM;
    }
    return LPCG_OK;
}

}  // namespace
}  // namespace lpcg

extern "C" int lpcg_gnn_predict_x0(const lpcg_system *s, const lpcg_gnn *net, const double *b, void *ws,
                                   int64_t ws_bytes, float *l_val, float *ut_val, double *x0, hipStream_t st) {
    int rc = check_head(s, net, ws, ws_bytes, "lpcg_gnn_predict_x0");
    if (rc) return rc;
    if (!x0) {
        set_error("lpcg_gnn_predict_x0: x0 is NULL");
        return LPCG_EINVAL;
    }
    if ((rc = gnn_forward(s, net, b, ws, ws_bytes, false, l_val, ut_val, st))) return rc;
    const GnnWs L = gnn_ws_layout(s, net->h, net->n_mp, false);
    const unsigned char *w = (const unsigned char *)ws;
    double *dst = s->perm ? s->xperm : x0;
    k_x0_scale<<<nblk(s->n, 256), 256, 0, st>>>(s->n, s->row_sys, (const double *)(w + L.sys_s),
                                                (const double *)(w + L.sys_rms), (const float *)(w + L.xhat), dst);
    LPCG_LAUNCH_CHECK();
    return s->perm ? from_internal_f64(s, s->xperm, x0, st) : LPCG_OK;
}

extern "C" int lpcg_x0_loss(const lpcg_system *s, const lpcg_gnn *net, void *ws, int64_t ws_bytes,
                            const double *x, double weight, double *loss, hipStream_t st) {
    int rc = check_head(s, net, ws, ws_bytes, "lpcg_x0_loss");
    if (rc) return rc;
    if (!x || !loss) {
        set_error("lpcg_x0_loss: invalid arguments");
        return LPCG_EINVAL;
    }
    if (s->perm) {
        if ((rc = to_internal_f64(s, x, s->xperm, st))) return rc;
        x = s->xperm;
    }
    const GnnWs L = gnn_ws_layout(s, net->h, net->n_mp, false);
    unsigned char *w = (unsigned char *)ws;
    const int nseg = norm_segments(s);
    double *part = (double *)(w + L.norm_part);
    k_x0_loss_part<<<dim3(nseg, s->nsys), kGnnThreads, 0, st>>>(
        nseg, s->sys_rowptr, (const double *)(w + L.sys_s), (const double *)(w + L.sys_rms),
        (const float *)(w + L.xhat), x, weight, weight != 0.0 ? (float *)(w + L.gxhat) : nullptr, part);
    k_x0_loss_fin<<<nblk(s->nsys, 64), 64, 0, st>>>(s->nsys, nseg, part, loss);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

// ===========================================================================
// Reverse mode of the network (hand-written).  For every Linear layer
// y = x W + b the data gradient gx = g W^T runs on MFMA with W staged
// untransposed; weight gradients dW = X^T G and bias gradients sum(G) are
// reductions over all rows done by one generic kernel (k_wgrad) into
// per-block partials, summed in a fixed order at the end (no atomics: the
// gradient is bit-reproducible).  Forward pre-activations are recomputed from
// the BF16 activations kept by the training forward.
// ===========================================================================
namespace lpcg {
namespace {

__device__ __forceinline__ float sigmoid_f(float x) { return 1.f / (1.f + expf(-x)); }

// d loss / d d_k from d loss / d L (pair average; softplus diagonal and sqrt(s)
// in mode 0; sqrt(A_jj) column scale with a fixed diagonal in mode 1 or the
// shifted-softplus diagonal in mode 2).
__global__ void k_assemble_bwd(int nnz, int mode, const int *__restrict__ rowptr, const int *__restrict__ lrowptr,
                               const int *__restrict__ erow, const int *__restrict__ col,
                               const int *__restrict__ rev, const int *__restrict__ row_sys,
                               const double *__restrict__ sys_s, const double *__restrict__ diag64,
                               const float *__restrict__ d, const float *__restrict__ gl, float *__restrict__ gd) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int i = erow[k], j = col[k];
    float g;
    if (i == j) {
        const int p = lrowptr[i] + (k - rowptr[i]);
        if (mode == 0) {
            const float sq = (float)sqrt(sys_s[row_sys[i]]);
            g = softplus_f(d[k]) > 1e-6f ? sq * gl[p] * sigmoid_f(d[k]) : 0.f;
        } else if (mode == 2) {
            const float ds = d[k] + kDiagShift;
            g = softplus_f(ds) > 1e-6f ? (float)sqrt(diag64[i]) * gl[p] * sigmoid_f(ds) : 0.f;
        } else {
            g = 0.f;
        }
    } else {
        // the lower entry of the pair: (i, j) if i > j, else (j, i)
        const int lo_r = i > j ? i : j, lo_c = i > j ? j : i;
        const int klo = i > j ? k : rev[k];
        const int p = lrowptr[lo_r] + (klo - rowptr[lo_r]);
        const float scale = mode == 0 ? (float)sqrt(sys_s[row_sys[i]]) : (float)sqrt(diag64[lo_c]);
        float gp = gl[p];
        if (mode == 3) {  // through the completed diagonal: dL_ii / dL_ij = -L_ij / L_ii
            const double rad = complete_radicand(lo_r, rowptr, lrowptr, col, rev, diag64, d);
            if (rad > kCompleteFloor * diag64[lo_r]) {
                const float lij = scale * (0.5f * (d[klo] + d[rev[klo]]));
                gp -= gl[lrowptr[lo_r + 1] - 1] * lij / (float)sqrt(rad);
            }
        }
        g = 0.5f * scale * gp;
    }
    gd[k] = g;
}

// Decoder MLP h -> h -> 1 on `nnz` rows of ET (the edge decoder on E_T, or
// the initial-guess head on V_T): pre = ET Wd0 + bd0, d = relu(pre) wd1 + bd1.
// Writes the hidden activation HD, its gradient GHD and d loss / d ET.
template <int H>
__global__ void __launch_bounds__(kGnnThreads) k_dec_bwd(int nnz, const float *__restrict__ P, MlpOff md,
                                                         const __bf16 *__restrict__ ET,
                                                         const float *__restrict__ gd, __bf16 *__restrict__ HD,
                                                         float *__restrict__ GHD, float *__restrict__ gE) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __bf16 wd[H * H], wdT[H * H];
    stage_weights<false>(wd, P + md.W0, H, H, H);
    stage_weightsT<true>(wdT, P + md.W0, H, H, H);
    __syncthreads();
    const int lane = lane_id();
    const float *w1d = P + md.W1;
    const int ntiles = (nnz + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int e = tile * 32 + (lane & 31);
        const bool valid = e < nnz;
        f32x16 pre[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) pre[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            bf16x8 b;
            if (valid) {
                b = load8(ET + (size_t)e * H + k_nat(s, 0, lane));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = (__bf16)0.f;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) pre[mt] = mfma(lds_op(wd, S, mt, s, lane), b, pre[mt]);
        }
        add_bias<MT>(pre, P + md.b0, lane, false);
        const float ge = valid ? gd[e] : 0.f;
        f32x16 hd[MT], g[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float v = pre[mt][i];
                hd[mt][i] = fmaxf(v, 0.f);
                g[mt][i] = v > 0.f ? ge * w1d[acc_feat(mt, i, lane)] : 0.f;
            }
        f32x16 gx[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) gx[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8 b = acc_operand<MT>(g, s);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) gx[mt] = mfma(lds_op(wdT, S, mt, s, lane), b, gx[mt]);
        }
        if (valid) {
            store_acc_bf16<MT>(HD + (size_t)e * H, hd, lane);
            store_acc_f32<MT>(GHD + (size_t)e * H, g, lane);
            store_acc_f32<MT>(gE + (size_t)e * H, gx, lane);
        }
    }
}

// Edge layer t: recompute g1 = relu(E_t We + Pa[r] + Pb[c] + b0); from
// gEn = d loss / d E_{t+1}: GH = (gEn W1^T) * [g1 > 0], gEt = GH We^T.
template <int H>
__global__ void __launch_bounds__(kGnnThreads) k_edge_bwd(int nnz, const int *__restrict__ erow,
                                                          const int *__restrict__ col,
                                                          const float *__restrict__ P, MlpOff me,
                                                          const __bf16 *__restrict__ Et,
                                                          const __bf16 *__restrict__ Pa,
                                                          const __bf16 *__restrict__ Pb,
                                                          const float *__restrict__ gEn, __bf16 *__restrict__ G1,
                                                          float *__restrict__ GH, float *__restrict__ gEt) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __bf16 we[H * H], w1T[H * H], weT[H * H];
    stage_weights<false>(we, P + me.W0, H, H, H);
    stage_weightsT<false>(w1T, P + me.W1, H, H, H);
    stage_weightsT<true>(weT, P + me.W0, H, H, H);
    __syncthreads();
    const int lane = lane_id();
    const float *b0 = P + me.b0;
    const int ntiles = (nnz + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int e = tile * 32 + (lane & 31);
        const bool valid = e < nnz;
        const int r = valid ? erow[e] : 0, c = valid ? col[e] : 0;
        f32x16 pre[MT], gg[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            pre[mt] = zero16();
            gg[mt] = zero16();
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            bf16x8 bx, bg;
            if (valid) {
                bx = load8(Et + (size_t)e * H + k_nat(s, 0, lane));
                bg = load8f(gEn + (size_t)e * H + k_nat(s, 0, lane));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    bx[j] = (__bf16)0.f;
                    bg[j] = (__bf16)0.f;
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                pre[mt] = mfma(lds_op(we, S, mt, s, lane), bx, pre[mt]);
                gg[mt] = mfma(lds_op(w1T, S, mt, s, lane), bg, gg[mt]);
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = acc_feat(mt, 4 * q, lane);
                bf16x4 ga, gb;
                if (valid) {
                    ga = *reinterpret_cast<const bf16x4 *>(Pa + (size_t)r * H + f);
                    gb = *reinterpret_cast<const bf16x4 *>(Pb + (size_t)c * H + f);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float add = valid ? (float)ga[t] + (float)gb[t] : 0.f;
                    const float v = pre[mt][4 * q + t] + add + b0[f + t];
                    pre[mt][4 * q + t] = fmaxf(v, 0.f);
                    if (!(v > 0.f)) gg[mt][4 * q + t] = 0.f;
                }
            }
        f32x16 gx[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) gx[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8 b = acc_operand<MT>(gg, s);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) gx[mt] = mfma(lds_op(weT, S, mt, s, lane), b, gx[mt]);
        }
        if (valid) {
            store_acc_bf16<MT>(G1 + (size_t)e * H, pre, lane);
            store_acc_f32<MT>(GH + (size_t)e * H, gg, lane);
            store_acc_f32<MT>(gEt + (size_t)e * H, gx, lane);
        }
    }
}

// Node layer t.  From GH (edge hidden gradients): gPa_i = sum_{k in row i}
// GH[k], gPb_j = sum_{k in row j} GH[rev k]; gVn = gVacc + gPa Wa^T + gPb Wb^T
// (d loss / d V_{t+1}); node MLP: recompute X = [V_t, m_t], h1 = relu(X W0 +
// b0); GH1 = (gVn W1^T) * [h1 > 0]; [gVmlp, gm] = GH1 W0^T.
template <int H>
__global__ void __launch_bounds__(kGnnThreads) k_node_bwd(
    int n, const int *__restrict__ rowptr, const int *__restrict__ col, const int *__restrict__ rev,
    const float *__restrict__ P, MlpOff mv, MlpOff me, const __bf16 *__restrict__ Vt,
    const __bf16 *__restrict__ Et, const float *__restrict__ GH, const float *__restrict__ gVacc,
    float *__restrict__ gPa, float *__restrict__ gPb, __bf16 *__restrict__ H1, float *__restrict__ GVN,
    float *__restrict__ GH1, __bf16 *__restrict__ Mt, float *__restrict__ gm, float *__restrict__ gVmlp) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __bf16 w0[2 * H * H], waT[H * H], wbT[H * H], w1T[H * H], w0T[2 * H * H];
    stage_weights<false>(w0, P + mv.W0, H, 2 * H, H);
    stage_weightsT<false>(waT, P + me.W0 + H * H, H, H, H);
    stage_weightsT<false>(wbT, P + me.W0 + 2 * H * H, H, H, H);
    stage_weightsT<true>(w1T, P + mv.W1, H, H, H);
    stage_weightsT<true>(w0T, P + mv.W0, H, H, 2 * H);
    __syncthreads();
    const int lane = lane_id();
    const int ntiles = (n + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int i = tile * 32 + (lane & 31);
        const bool valid = i < n;
        // gPa, gPb in natural order; B operands of the projection gradients
        f32x16 gvn[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) gvn[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            float sa[8], sb[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) sa[j] = sb[j] = 0.f;
            if (valid) {
                const int f = k_nat(s, 0, lane);
                for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                    const float *ga = GH + (size_t)k * H + f;
                    const float *gb = GH + (size_t)rev[k] * H + f;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        sa[j] += ga[j];
                        sb[j] += gb[j];
                    }
                }
                float *oa = gPa + (size_t)i * H + f, *ob = gPb + (size_t)i * H + f;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    oa[j] = sa[j];
                    ob[j] = sb[j];
                }
            }
            bf16x8 ba, bb;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                ba[j] = (__bf16)sa[j];
                bb[j] = (__bf16)sb[j];
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                gvn[mt] = mfma(lds_op(waT, S, mt, s, lane), ba, gvn[mt]);
                gvn[mt] = mfma(lds_op(wbT, S, mt, s, lane), bb, gvn[mt]);
            }
        }
        if (valid && gVacc) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const f32x4 v = *reinterpret_cast<const f32x4 *>(gVacc + (size_t)i * H + acc_feat(mt, 4 * q, lane));
#pragma unroll
                    for (int t = 0; t < 4; ++t) gvn[mt][4 * q + t] += v[t];
                }
        }
        // recompute the node MLP input and hidden layer
        bf16x8 bx[2 * S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (valid) {
                bx[s] = load8(Vt + (size_t)i * H + k_nat(s, 0, lane));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) bx[s][j] = (__bf16)0.f;
            }
        }
        float msum[S][8];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) msum[s][j] = 0.f;
        if (valid) {
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int c = col[k];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const bf16x8 e8 = load8(Et + (size_t)k * H + k_nat(s, 0, lane));
                    const bf16x8 v8 = load8(Vt + (size_t)c * H + k_nat(s, 0, lane));
#pragma unroll
                    for (int j = 0; j < 8; ++j) msum[s][j] += (float)e8[j] * (float)v8[j];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int j = 0; j < 8; ++j) bx[S + s][j] = (__bf16)msum[s][j];
            if (valid) *reinterpret_cast<bf16x8 *>(Mt + (size_t)i * H + k_nat(s, 0, lane)) = bx[S + s];
        }
        f32x16 h1[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) h1[mt] = zero16();
#pragma unroll
        for (int s = 0; s < 2 * S; ++s)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) h1[mt] = mfma(lds_op(w0, 2 * S, mt, s, lane), bx[s], h1[mt]);
        add_bias<MT>(h1, P + mv.b0, lane, false);
        f32x16 gh1[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) gh1[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8 b = acc_operand<MT>(gvn, s);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) gh1[mt] = mfma(lds_op(w1T, S, mt, s, lane), b, gh1[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const bool on = h1[mt][q] > 0.f;
                h1[mt][q] = on ? h1[mt][q] : 0.f;
                if (!on) gh1[mt][q] = 0.f;
            }
        f32x16 gx[2 * MT];
#pragma unroll
        for (int mt = 0; mt < 2 * MT; ++mt) gx[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8 b = acc_operand<MT>(gh1, s);
#pragma unroll
            for (int mt = 0; mt < 2 * MT; ++mt) gx[mt] = mfma(lds_op(w0T, S, mt, s, lane), b, gx[mt]);
        }
        if (valid) {
            store_acc_f32<MT>(GVN + (size_t)i * H, gvn, lane);
            store_acc_bf16<MT>(H1 + (size_t)i * H, h1, lane);
            store_acc_f32<MT>(GH1 + (size_t)i * H, gh1, lane);
            f32x16 gv[MT], gmm[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                gv[mt] = gx[mt];
                gmm[mt] = gx[MT + mt];
            }
            store_acc_f32<MT>(gVmlp + (size_t)i * H, gv, lane);
            store_acc_f32<MT>(gm + (size_t)i * H, gmm, lane);
        }
    }
}

// Adjoint of m_i = sum_{k in row i} E[k] * V[col k] with respect to E:
// gE[k] += gm[row k] * V[col k].
template <int H>
__global__ void k_agg_bwd_edge(int nnz, const int *__restrict__ erow, const int *__restrict__ col,
                               const __bf16 *__restrict__ V, const float *__restrict__ gm, float *__restrict__ gE) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nnz * (H / 4)) return;
    const int e = (int)(idx / (H / 4)), f = (int)(idx % (H / 4)) * 4;
    const int r = erow[e], c = col[e];
    f32x4 g = *reinterpret_cast<f32x4 *>(gE + (size_t)e * H + f);
    const f32x4 m = *reinterpret_cast<const f32x4 *>(gm + (size_t)r * H + f);
    const bf16x4 v = *reinterpret_cast<const bf16x4 *>(V + (size_t)c * H + f);
#pragma unroll
    for (int t = 0; t < 4; ++t) g[t] += m[t] * (float)v[t];
    *reinterpret_cast<f32x4 *>(gE + (size_t)e * H + f) = g;
}

// ... and with respect to V: gV[j] = gVmlp[j] + sum_{k in row j} gm[col k] * E[rev k]
// (the entries (i, j) with col = j are the reverses of row j's entries).
template <int H>
__global__ void k_agg_bwd_node(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                               const int *__restrict__ rev, const __bf16 *__restrict__ E,
                               const float *__restrict__ gm, const float *__restrict__ gVmlp,
                               float *__restrict__ gV) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * (H / 4)) return;
    const int j = (int)(idx / (H / 4)), f = (int)(idx % (H / 4)) * 4;
    f32x4 g = *reinterpret_cast<const f32x4 *>(gVmlp + (size_t)j * H + f);
    for (int k = rowptr[j]; k < rowptr[j + 1]; ++k) {
        const f32x4 m = *reinterpret_cast<const f32x4 *>(gm + (size_t)col[k] * H + f);
        const bf16x4 e = *reinterpret_cast<const bf16x4 *>(E + (size_t)rev[k] * H + f);
#pragma unroll
        for (int t = 0; t < 4; ++t) g[t] += m[t] * (float)e[t];
    }
    *reinterpret_cast<f32x4 *>(gV + (size_t)j * H + f) = g;
}

// Encoder: h = relu(x W0 + b0) (kept as Henc), GHenc = (gOut W1^T) * [h > 0],
// Xs = x.
template <int H>
__global__ void __launch_bounds__(kGnnThreads) k_enc_bwd(int rows, const float *__restrict__ P, MlpOff m,
                                                         const float *__restrict__ xs,
                                                         const float *__restrict__ gOut, __bf16 *__restrict__ Henc,
                                                         float *__restrict__ GHenc) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __bf16 w1T[H * H];
    stage_weightsT<false>(w1T, P + m.W1, H, H, H);
    __syncthreads();
    const int lane = lane_id();
    const float *W0 = P + m.W0, *b0 = P + m.b0;
    const int ntiles = (rows + 31) / 32;
    for (int tile = blockIdx.x * 4 + threadIdx.x / kWave; tile < ntiles; tile += gridDim.x * 4) {
        const int r = tile * 32 + (lane & 31);
        const bool valid = r < rows;
        const float x = valid ? xs[r] : 0.f;
        f32x16 gh[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) gh[mt] = zero16();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            bf16x8 hb, gb;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = k_nat(s, j, lane);
                hb[j] = (__bf16)fmaxf(x * W0[k] + b0[k], 0.f);
            }
            if (valid) {
                *reinterpret_cast<bf16x8 *>(Henc + (size_t)r * H + k_nat(s, 0, lane)) = hb;
                gb = load8f(gOut + (size_t)r * H + k_nat(s, 0, lane));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) gb[j] = (__bf16)0.f;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) gh[mt] = mfma(lds_op(w1T, S, mt, s, lane), gb, gh[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int f = acc_feat(mt, i, lane);
                if (!(x * W0[f] + b0[f] > 0.f)) gh[mt][i] = 0.f;
            }
        if (valid) store_acc_f32<MT>(GHenc + (size_t)r * H, gh, lane);
    }
}

// Sources of the weight-gradient reduction dW = X^T G (rows x K each).
enum SrcKind : int { SRC_BF16 = 0, SRC_F32 = 1, SRC_SCALAR = 2, SRC_BF16_CAT = 3 };
struct WSrc {
    int kind;
    const void *a;  // matrix / scalar vector / first half of a concatenation
    const void *b;  // second half (SRC_BF16_CAT), same width as the first
    int K;          // columns (1 for scalars; total width for concatenations)
};

__device__ __forceinline__ float src_at(const WSrc &s, int row, int c) {
    switch (s.kind) {
        case SRC_BF16: return (float)((const __bf16 *)s.a)[(size_t)row * s.K + c];
        case SRC_F32: return ((const float *)s.a)[(size_t)row * s.K + c];
        case SRC_SCALAR: return c == 0 ? ((const float *)s.a)[row] : 0.f;
        default: {
            const int half = s.K / 2;
            return c < half ? (float)((const __bf16 *)s.a)[(size_t)row * half + c]
                            : (float)((const __bf16 *)s.b)[(size_t)row * half + (c - half)];
        }
    }
}

// Per-block partial of dW = X^T G (and sum(G) for the bias) over the rows.
// Each wave stages 32-row tiles transposed in its own LDS slice and
// accumulates on MFMA with the rows as the contraction; the block's 4 waves
// are summed in a fixed order.  KXP / MP: K of X and G padded to 32.
template <int KXP, int MP>
__global__ void __launch_bounds__(kGnnThreads) k_wgrad(int rows, WSrc X, WSrc G, int Mreal,
                                                       float *__restrict__ wpart, int ptotal, int offW,
                                                       int offB) {
    constexpr int KT = KXP / 32, MTN = MP / 32;
    __shared__ __bf16 xt[4][KXP * 32];
    __shared__ __bf16 gt[4][MP * 32];
    __shared__ float red[4][32 * 32];
    __shared__ float bred[4][64];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    f32x16 acc[KT][MTN];
#pragma unroll
    for (int a = 0; a < KT; ++a)
#pragma unroll
        for (int b = 0; b < MTN; ++b) acc[a][b] = zero16();
    float bsum = 0.f;
    const int ntiles = (rows + 31) / 32;
    for (int tile = blockIdx.x * 4 + w; tile < ntiles; tile += gridDim.x * 4) {
        for (int idx = lane; idx < 32 * KXP; idx += kWave) {
            const int r = idx / KXP, c = idx % KXP;
            const int row = tile * 32 + r;
            const float v = (row < rows && c < X.K) ? src_at(X, row, c) : 0.f;
            xt[w][c * 32 + r] = (__bf16)v;
        }
        for (int idx = lane; idx < 32 * MP; idx += kWave) {
            const int r = idx / MP, c = idx % MP;
            const int row = tile * 32 + r;
            const float v = (row < rows && c < G.K) ? src_at(G, row, c) : 0.f;
            gt[w][c * 32 + r] = (__bf16)v;
            bsum += v;  // column c = lane % MP for this lane, fixed
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int a = 0; a < KT; ++a) {
                const bf16x8 av =
                    *reinterpret_cast<const bf16x8 *>(&xt[w][(a * 32 + (lane & 31)) * 32 + s * 16 + 8 * (lane >> 5)]);
#pragma unroll
                for (int b = 0; b < MTN; ++b) {
                    const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(
                        &gt[w][(b * 32 + (lane & 31)) * 32 + s * 16 + 8 * (lane >> 5)]);
                    acc[a][b] = mfma(av, bv, acc[a][b]);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // fixed-order sum over the block's waves, one 32x32 tile at a time
    for (int a = 0; a < KT; ++a)
        for (int b = 0; b < MTN; ++b) {
#pragma unroll
            for (int i = 0; i < 16; ++i) red[w][(8 * (i >> 2) + 4 * (lane >> 5) + (i & 3)) * 32 + (lane & 31)] = acc[a][b][i];
            __syncthreads();
            for (int e = threadIdx.x; e < 32 * 32; e += kGnnThreads) {
                const float v = red[0][e] + red[1][e] + red[2][e] + red[3][e];
                const int kx = a * 32 + e / 32, m = b * 32 + e % 32;
                if (kx < X.K && m < Mreal) wpart[(size_t)blockIdx.x * ptotal + offW + (size_t)kx * Mreal + m] = v;
            }
            __syncthreads();
        }
    if (offB >= 0) {
        if (MP == 32) bsum += __shfl_xor(bsum, 32, kWave);
        if (lane < MP) bred[w][lane] = bsum;
        __syncthreads();
        if (threadIdx.x < Mreal)
            wpart[(size_t)blockIdx.x * ptotal + offB + threadIdx.x] =
                bred[0][threadIdx.x] + bred[1][threadIdx.x] + bred[2][threadIdx.x] + bred[3][threadIdx.x];
    }
}

__global__ void k_wreduce(int ptotal, int nb, const float *__restrict__ wpart, float *__restrict__ dparams) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ptotal) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += wpart[(size_t)b * ptotal + i];
    dparams[i] = s;
}

template <int KXP, int MP>
void wgrad(int rows, WSrc X, WSrc G, int Mreal, float *wpart, int ptotal, int offW, int offB, hipStream_t st) {
    k_wgrad<KXP, MP><<<kWgradBlocks, kGnnThreads, 0, st>>>(rows, X, G, Mreal, wpart, ptotal, offW, offB);
}

template <int H>
int backward_impl(const lpcg_system *s, const lpcg_gnn *net, unsigned char *ws, const GnnWs &L,
                  const float *dl, float *dparams, hipStream_t st) {
    const int T = net->n_mp;
    const GnnOff o = gnn_offsets(H, T, net->x_head != 0);
    const float *P = net->params;
    auto V = [&](int t) { return (const __bf16 *)(ws + L.V[t]); };
    auto E = [&](int t) { return (const __bf16 *)(ws + L.E[t]); };
    auto F = [&](size_t off) { return (float *)(ws + off); };
    auto B16 = [&](size_t off) { return (__bf16 *)(ws + off); };
    const double *sys_s = (const double *)(ws + L.sys_s), *sys_rms = (const double *)(ws + L.sys_rms);
    float *wpart = F(L.wpart);
    const int n = s->n, nnz = s->nnz, pt = o.total;
    auto bf = [](const void *p, int K) { return WSrc{SRC_BF16, p, nullptr, K}; };
    auto f32 = [](const void *p, int K) { return WSrc{SRC_F32, p, nullptr, K}; };
    auto sc = [](const void *p) { return WSrc{SRC_SCALAR, p, nullptr, 1}; };

    k_assemble_bwd<<<nblk(nnz, 256), 256, 0, st>>>(nnz, net->diag_mode, s->rowptr, s->lrowptr, s->erow,
                                                    s->colind, s->rev, s->row_sys, sys_s, s->diag64, F(L.d), dl,
                                                    F(L.gd));
    k_dec_bwd<H><<<gnn_blocks(nnz), kGnnThreads, 0, st>>>(nnz, P, o.dec, E(T), F(L.gd), B16(L.HD), F(L.GHD),
                                                          F(L.gE[T & 1]));
    wgrad<H, H>(nnz, bf(E(T), H), f32(F(L.GHD), H), H, wpart, pt, o.dec.W0, o.dec.b0, st);
    wgrad<H, 32>(nnz, bf(B16(L.HD), H), sc(F(L.gd)), 1, wpart, pt, o.dec.W1, o.dec.b1, st);
    const float *gVacc = nullptr;
    if (net->x_head) {
        // initial-guess head: same MLP shape as the edge decoder, on the node
        // latents V_T; its input gradient seeds d loss / d V_T (HD and GHD are
        // free again once the edge decoder's weight gradients are enqueued)
        float *gVT = F(L.gV[T & 1]);
        k_dec_bwd<H><<<gnn_blocks(n), kGnnThreads, 0, st>>>(n, P, o.xdec, V(T), F(L.gxhat), B16(L.HD),
                                                             F(L.GHD), gVT);
        wgrad<H, H>(n, bf(V(T), H), f32(F(L.GHD), H), H, wpart, pt, o.xdec.W0, o.xdec.b0, st);
        wgrad<H, 32>(n, bf(B16(L.HD), H), sc(F(L.gxhat)), 1, wpart, pt, o.xdec.W1, o.xdec.b1, st);
        gVacc = gVT;
    }
    for (int t = T - 1; t >= 0; --t) {
        float *gEn = F(L.gE[(t + 1) & 1]), *gEt = F(L.gE[t & 1]);
        k_edge_bwd<H><<<gnn_blocks(nnz), kGnnThreads, 0, st>>>(nnz, s->erow, s->colind, P, o.edge[t], E(t),
                                                               (const __bf16 *)(ws + L.Pa[t]),
                                                               (const __bf16 *)(ws + L.Pb[t]), gEn, B16(L.G1),
                                                               F(L.GH), gEt);
        wgrad<H, H>(nnz, bf(B16(L.G1), H), f32(gEn, H), H, wpart, pt, o.edge[t].W1, o.edge[t].b1, st);
        wgrad<H, H>(nnz, bf(E(t), H), f32(F(L.GH), H), H, wpart, pt, o.edge[t].W0, o.edge[t].b0, st);
        k_node_bwd<H><<<gnn_blocks(n), kGnnThreads, 0, st>>>(
            n, s->rowptr, s->colind, s->rev, P, o.node[t], o.edge[t], V(t), E(t), F(L.GH), gVacc, F(L.gPa),
            F(L.gPb), B16(L.H1), F(L.GVN), F(L.GH1), B16(L.Mt), F(L.gm), F(L.gVmlp));
        wgrad<H, H>(n, bf(V(t + 1), H), f32(F(L.gPa), H), H, wpart, pt, o.edge[t].W0 + H * H, -1, st);
        wgrad<H, H>(n, bf(V(t + 1), H), f32(F(L.gPb), H), H, wpart, pt, o.edge[t].W0 + 2 * H * H, -1, st);
        wgrad<H, H>(n, bf(B16(L.H1), H), f32(F(L.GVN), H), H, wpart, pt, o.node[t].W1, o.node[t].b1, st);
        wgrad<2 * H, H>(n, WSrc{SRC_BF16_CAT, V(t), B16(L.Mt), 2 * H}, f32(F(L.GH1), H), H, wpart, pt,
                        o.node[t].W0, o.node[t].b0, st);
        k_agg_bwd_edge<H><<<nblk((long)nnz * (H / 4), 256), 256, 0, st>>>(nnz, s->erow, s->colind, V(t), F(L.gm),
                                                                          gEt);
        float *gVout = F(L.gV[t & 1]);
        k_agg_bwd_node<H><<<nblk((long)n * (H / 4), 256), 256, 0, st>>>(n, s->rowptr, s->colind, s->rev, E(t),
                                                                        F(L.gm), F(L.gVmlp), gVout);
        gVacc = gVout;
    }
    // encoders: node (gradient gVacc w.r.t. V_0), edge (gE[0] w.r.t. E_0)
    k_enc_bwd<H><<<gnn_blocks(n), kGnnThreads, 0, st>>>(n, P, o.node_enc, F(L.Xn), gVacc, B16(L.Henc),
                                                         F(L.GHenc));
    wgrad<H, H>(n, bf(B16(L.Henc), H), f32(gVacc, H), H, wpart, pt, o.node_enc.W1, o.node_enc.b1, st);
    wgrad<32, H>(n, sc(F(L.Xn)), f32(F(L.GHenc), H), H, wpart, pt, o.node_enc.W0, o.node_enc.b0, st);
    k_enc_bwd<H><<<gnn_blocks(nnz), kGnnThreads, 0, st>>>(nnz, P, o.edge_enc, F(L.Xe), F(L.gE[0]), B16(L.Henc),
                                                           F(L.GHenc));
    wgrad<H, H>(nnz, bf(B16(L.Henc), H), f32(F(L.gE[0]), H), H, wpart, pt, o.edge_enc.W1, o.edge_enc.b1, st);
    wgrad<32, H>(nnz, sc(F(L.Xe)), f32(F(L.GHenc), H), H, wpart, pt, o.edge_enc.W0, o.edge_enc.b0, st);
    k_wreduce<<<nblk(pt, 256), 256, 0, st>>>(pt, kWgradBlocks, wpart, dparams);
    (void)sys_rms;
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

}  // namespace
}  // namespace lpcg

using namespace lpcg;

extern "C" int lpcg_gnn_backward(const lpcg_system *s, const lpcg_gnn *net, void *ws, int64_t ws_bytes,
                                 const float *dl_val, float *dparams, hipStream_t st) {
    int rc = check_net(net);
    if (rc) return rc;
    if (!s || !ws || !dl_val || !dparams) {
        set_error("lpcg_gnn_backward: invalid arguments");
        return LPCG_EINVAL;
    }
    const GnnWs L = gnn_ws_layout(s, net->h, net->n_mp, true);
    if ((size_t)ws_bytes < L.total) {
        set_error("lpcg_gnn_backward: workspace of %lld bytes, %zu needed", (long long)ws_bytes, L.total);
        return LPCG_ENOMEM;
    }
    if (net->h == 32) return backward_impl<32>(s, net, (unsigned char *)ws, L, dl_val, dparams, st);
    return backward_impl<64>(s, net, (unsigned char *)ws, L, dl_val, dparams, st);
}
