// Preconditioner GNN, forward (Method "Architecture"; technical-details
// appendix): encoders, n_mp message-passing layers, decoder, and the
// lower-triangular assembly L_ij = sqrt(s) (d_ij + d_ji)/2, L_ii =
// sqrt(s) max(softplus(d_ii), 1e-6).
//
// Kernels (H = latent width, 32 or 64; one wave = 32 rows, BF16 MFMA with
// FP32 accumulation, see kern_gnn.h):
//   k_gnn_norm   per system: s = mean(diag A), rms(b)
//   k_enc<NODE>  node encoder on b_i/rms, edge encoder on A_ij/s
//   k_node       aggregation m_i = sum_{k in row i} E[k] * V[col k] (fused),
//                node MLP on [V_i, m_i], and the projections V W_a, V W_b of
//                the edge MLP's first layer (factored: [e, v_i, v_j] W =
//                e W_e + (V W_a)[i] + (V W_b)[j])
//   k_edge<LAST> edge MLP per directed edge; the last layer also runs the
//                decoder and writes the scalar d per edge
//   k_assemble   pair average, softplus diagonal, sqrt(s) scaling
#include <algorithm>
#include <cstring>

#include "device_util.h"
#include "kern_gnn.h"
#include "lpcg_internal.h"

namespace lpcg {

GnnOff gnn_offsets(int h, int n_mp) {
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
    o.total = p;
    return o;
}

// Workspace layout (byte offsets, 256-byte aligned).
struct GnnWs {
    size_t sys_s, sys_rms;
    size_t V[kMaxMp + 1], Pa[kMaxMp], Pb[kMaxMp], E[kMaxMp + 1];
    size_t d;
    // backward scratch
    size_t gd, gE[2], gV[2], gH, gPa, gPb, wpart;
    size_t total;
};

// Waves that keep private weight-gradient partials in the backward pass.
int gnn_wpart_waves(const lpcg_system *s) {
    (void)s;
    return 1024;
}

GnnWs gnn_ws_layout(const lpcg_system *s, int h, int n_mp, bool train) {
    GnnWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t n = s->n, nnz = s->nnz;
    w.sys_s = take(sizeof(double) * s->nsys);
    w.sys_rms = take(sizeof(double) * s->nsys);
    const int nv = train ? n_mp + 1 : 2;
    const int np = train ? n_mp : 1;
    for (int i = 0; i < nv; ++i) w.V[i] = take(2 * n * h);
    for (int i = 0; i < np; ++i) {
        w.Pa[i] = take(2 * n * h);
        w.Pb[i] = take(2 * n * h);
    }
    for (int i = 0; i < nv; ++i) w.E[i] = take(2 * nnz * h);
    w.d = take(4 * nnz);
    if (train) {
        w.gd = take(4 * nnz);
        w.gE[0] = take(4 * nnz * h);
        w.gE[1] = take(4 * nnz * h);
        w.gV[0] = take(4 * n * h);
        w.gV[1] = take(4 * n * h);
        w.gH = take(4 * nnz * h);
        w.gPa = take(4 * n * h);
        w.gPb = take(4 * n * h);
        const GnnOff o = gnn_offsets(h, n_mp);
        w.wpart = take(sizeof(float) * (size_t)o.total * gnn_wpart_waves(s));
    }
    w.total = off;
    return w;
}

namespace {

constexpr int kGnnThreads = 256;  // 4 waves, 32 rows each per tile step
constexpr int kMaxGnnBlocks = 1024;

int nblk(long n, int t) { return (int)((n + t - 1) / t); }

__global__ void k_gnn_norm(int nsys, const int *__restrict__ sys_rowptr, const int *__restrict__ dpos,
                           const double *__restrict__ val, const double *__restrict__ b,
                           double *__restrict__ sys_s, double *__restrict__ sys_rms) {
    __shared__ double lds[kGnnThreads / kWave];
    const int sy = blockIdx.x;
    if (sy >= nsys) return;
    const int r0 = sys_rowptr[sy], r1 = sys_rowptr[sy + 1];
    double sd = 0, sb = 0;
    for (int i = r0 + threadIdx.x; i < r1; i += kGnnThreads) {
        sd += val[dpos[i]];
        sb += b[i] * b[i];
    }
    sd = block_sum<kGnnThreads>(sd, lds);
    sb = block_sum<kGnnThreads>(sb, lds);
    if (threadIdx.x == 0) {
        const double cnt = (double)(r1 - r0);
        sys_s[sy] = sd / cnt;
        const double rms = sqrt(sb / cnt);
        sys_rms[sy] = rms > 0 ? rms : 1.0;
    }
}

// Encoder: out[row] = relu(x W0 + b0) W1 + b1 with scalar input x.
template <int H, bool NODE>
__global__ void __launch_bounds__(kGnnThreads) k_enc(int rows, const float *__restrict__ P, MlpOff m,
                                                     const double *__restrict__ xin,
                                                     const int *__restrict__ erow,
                                                     const int *__restrict__ row_sys,
                                                     const double *__restrict__ sys_scale,
                                                     __bf16 *__restrict__ out) {
    constexpr int S = H / 16, MT = H / 32;
    __shared__ __bf16 w1[H * H];
    stage_weights<false>(w1, P + m.W1, H, H, H);
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
            x = (float)(xin[r] / sys_scale[row_sys[node]]);
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

__device__ __forceinline__ float softplus_f(float x) { return x > 20.f ? x : log1pf(expf(x)); }

// L value of the lower-pattern entry with A-position k.
__device__ __forceinline__ float l_entry(int k, const int *__restrict__ erow, const int *__restrict__ col,
                                         const int *__restrict__ rev, const int *__restrict__ row_sys,
                                         const double *__restrict__ sys_s, const float *__restrict__ d) {
    const int i = erow[k];
    const float sq = (float)sqrt(sys_s[row_sys[i]]);
    if (col[k] == i) return sq * fmaxf(softplus_f(d[k]), 1e-6f);
    return sq * 0.5f * (d[k] + d[rev[k]]);
}

__global__ void k_assemble(int nnz_l, const int *__restrict__ lsrc, const int *__restrict__ u2l,
                           const int *__restrict__ erow, const int *__restrict__ col,
                           const int *__restrict__ rev, const int *__restrict__ row_sys,
                           const double *__restrict__ sys_s, const float *__restrict__ d,
                           float *__restrict__ lval, float *__restrict__ utval) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz_l) return;
    if (lval) lval[p] = l_entry(lsrc[p], erow, col, rev, row_sys, sys_s, d);
    if (utval) utval[p] = l_entry(lsrc[u2l[p]], erow, col, rev, row_sys, sys_s, d);
}

int gnn_blocks(long rows) { return std::max(1, std::min(kMaxGnnBlocks, nblk(rows, 32 * 4))); }

template <int H>
int forward_impl(const lpcg_system *s, const lpcg_gnn *net, const double *b, unsigned char *ws,
                 const GnnWs &L, bool train, float *lval, float *utval, hipStream_t st) {
    const GnnOff o = gnn_offsets(H, net->n_mp);
    const float *P = net->params;
    double *sys_s = (double *)(ws + L.sys_s), *sys_rms = (double *)(ws + L.sys_rms);
    k_gnn_norm<<<s->nsys, kGnnThreads, 0, st>>>(s->nsys, s->sys_rowptr, s->dpos, s->val64, b, sys_s, sys_rms);
    auto V = [&](int t) { return (__bf16 *)(ws + L.V[train ? t : (t & 1)]); };
    auto E = [&](int t) { return (__bf16 *)(ws + L.E[train ? t : (t & 1)]); };
    auto Pa = [&](int t) { return (__bf16 *)(ws + L.Pa[train ? t : 0]); };
    auto Pb = [&](int t) { return (__bf16 *)(ws + L.Pb[train ? t : 0]); };
    float *d = (float *)(ws + L.d);
    k_enc<H, true><<<gnn_blocks(s->n), kGnnThreads, 0, st>>>(s->n, P, o.node_enc, b, s->erow, s->row_sys,
                                                              sys_rms, V(0));
    k_enc<H, false><<<gnn_blocks(s->nnz), kGnnThreads, 0, st>>>(s->nnz, P, o.edge_enc, s->val64, s->erow,
                                                                 s->row_sys, sys_s, E(0));
    const int T = net->n_mp;
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
    k_assemble<<<nblk(s->nnz_l, 256), 256, 0, st>>>(s->nnz_l, s->lsrc, s->u2l, s->erow, s->colind, s->rev,
                                                     s->row_sys, sys_s, d, lval, utval);
    LPCG_LAUNCH_CHECK();
    return LPCG_OK;
}

int check_net(const lpcg_gnn *net) {
    if (!net || !net->params || (net->h != 32 && net->h != 64) || net->n_mp < 1 || net->n_mp > kMaxMp) {
        set_error("gnn: h must be 32 or 64 and 1 <= n_mp <= %d", kMaxMp);
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
    const GnnWs L = gnn_ws_layout(s, net->h, net->n_mp, train);
    if ((size_t)ws_bytes < L.total) {
        set_error("gnn forward: workspace of %lld bytes, %zu needed", (long long)ws_bytes, L.total);
        return LPCG_ENOMEM;
    }
    if (net->h == 32) return forward_impl<32>(s, net, b, (unsigned char *)ws, L, train, lval, utval, st);
    return forward_impl<64>(s, net, b, (unsigned char *)ws, L, train, lval, utval, st);
}

}  // namespace lpcg

using namespace lpcg;

extern "C" int64_t lpcg_gnn_param_count(int32_t h, int32_t n_mp) {
    if (h <= 0 || n_mp < 1 || n_mp > kMaxMp) return -1;
    return gnn_offsets(h, n_mp).total;
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
