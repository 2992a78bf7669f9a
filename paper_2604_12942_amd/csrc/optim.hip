// Sparse Adam over component-major parameter groups, and the L1 colour / depth loss (Eq. 9,
// 10, 12 with the all-ones mask).  Both are streams over HBM: coalesced, one element per lane.
#include "gsr_internal.h"

namespace gsr {

__global__ void k_adam(gsr_adam_groups G, int64_t rows, const uint8_t *__restrict__ mask, float b1, float b2,
                       float eps, float bc1, float bc2) {
    const int gi = blockIdx.y;
    const int64_t numel = rows * G.cols[gi];
    float *__restrict__ p = G.param[gi];
    float *__restrict__ gr = G.grad[gi];
    float *__restrict__ m = G.m[gi];
    float *__restrict__ v = G.v[gi];
    const float lr = G.lr[gi];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < numel; e += (int64_t)gridDim.x * blockDim.x) {
        const float g = gr[e];
        const int64_t row = e % rows;
        if (!mask || mask[row]) {
            const float mm = b1 * m[e] + (1.0f - b1) * g;
            const float vv = b2 * v[e] + (1.0f - b2) * g * g;
            m[e] = mm;
            v[e] = vv;
            p[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
        }
        gr[e] = 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_loss_l1(const float *__restrict__ rgb, const float *__restrict__ depth,
                                                 const float *__restrict__ trgb, const float *__restrict__ tdepth,
                                                 const int32_t *__restrict__ tidx, int64_t P, int V, float lam,
                                                 float *__restrict__ grgb,
                                                 float *__restrict__ gdepth, double *__restrict__ loss) {
    __shared__ double s_red[4];
    const float invP = 1.0f / (float)P;
    double acc = 0.0;
    const int64_t total = (int64_t)V * P;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = e / P, pix = e % P;
        const int64_t slot = tidx ? (int64_t)tidx[v] : v;
        const int64_t base = v * 3 * P + pix, tbase = slot * 3 * P + pix;
        float l = 0.f;
        for (int ch = 0; ch < 3; ch++) {
            const float d = rgb[base + ch * P] - trgb[tbase + ch * P];
            l += fabsf(d);
            grgb[base + ch * P] = (d > 0.f ? invP : (d < 0.f ? -invP : 0.f));
        }
        float gd = 0.f;
        if (tdepth) {
            const float d = depth[e] - tdepth[slot * P + pix];
            l += lam * fabsf(d);
            gd = lam * (d > 0.f ? invP : (d < 0.f ? -invP : 0.f));
        }
        if (gdepth) gdepth[e] = gd;
        acc += (double)l;
    }
    acc = wave_sum_d(acc);
    if (__lane_id() == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, (s_red[0] + s_red[1] + s_red[2] + s_red[3]) / (double)P);
}

// Per-step preparation of the batched optimiser in one launch: the step's camera records
// gathered from the pool (96-byte records as 24 words), the view indices as int32, the loss sum
// cleared, the Adam step number advanced and the row mask cleared (16 bytes per store where the
// whole 16 lie inside).
__global__ void k_step_prep(const uint32_t *__restrict__ pool, int32_t n_pool, const int64_t *__restrict__ view_idx,
                            int32_t V, uint32_t *__restrict__ cams, int32_t *__restrict__ view_idx32,
                            double *__restrict__ loss, int32_t *__restrict__ step, uint8_t *__restrict__ row_mask,
                            int64_t n) {
    constexpr int kWords = (int)(sizeof(gsr_camera) / 4);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = tid; k < (int64_t)V * kWords; k += stride) {
        const int64_t v = k / kWords, w = k - v * kWords;
        const int64_t s = view_idx[v];
        if (s >= 0 && s < n_pool) cams[k] = pool[s * kWords + w];
    }
    if (view_idx32)
        for (int64_t v = tid; v < V; v += stride) view_idx32[v] = (int32_t)view_idx[v];
    if (tid == 0) {
        if (loss) *loss = 0.0;
        if (step) *step += 1;
    }
    if (row_mask) {
        const int64_t n16 = n / 16;
        uint4 *m16 = reinterpret_cast<uint4 *>(row_mask);
        for (int64_t i = tid; i < n16; i += stride) m16[i] = make_uint4(0u, 0u, 0u, 0u);
        for (int64_t i = n16 * 16 + tid; i < n; i += stride) row_mask[i] = 0;
    }
}

}  // namespace gsr

using namespace gsr;

extern "C" gsr_status gsr_step_prep_launch(const gsr_camera *pool, int32_t n_pool, const int64_t *view_idx, int32_t V,
                                           gsr_camera *cams, int32_t *view_idx32, double *loss, int32_t *step,
                                           uint8_t *row_mask, int64_t n, hipStream_t st) {
    static_assert(sizeof(gsr_camera) % 4 == 0, "camera records are whole words");
    const int64_t cam_words = (int64_t)V * (int64_t)(sizeof(gsr_camera) / 4);
    const int64_t mask_work = row_mask ? n / 16 : 0;
    const int64_t work = mask_work > cam_words ? mask_work : cam_words;
    const int nb = (int)(ceil_div(work, 256) < 1024 ? ceil_div(work, 256) : 1024);
    k_step_prep<<<nb, 256, 0, st>>>(reinterpret_cast<const uint32_t *>(pool), n_pool, view_idx, V,
                                    reinterpret_cast<uint32_t *>(cams), view_idx32, loss, step, row_mask, n);
    return last_launch();
}

extern "C" gsr_status gsr_adam_launch(const gsr_adam_groups *g, int64_t rows, const uint8_t *mask, float b1, float b2,
                                      float eps, int step, hipStream_t st) {
    int64_t maxcols = 0;
    for (int k = 0; k < g->n_groups; k++) maxcols = g->cols[k] > maxcols ? g->cols[k] : maxcols;
    const int64_t work = rows * maxcols;
    if (work == 0) return GSR_OK;
    const int nbx = (int)(ceil_div(work, 256) < 4096 ? ceil_div(work, 256) : 4096);
    const float bc1 = (float)(1.0 - pow((double)b1, step)), bc2 = (float)(1.0 - pow((double)b2, step));
    k_adam<<<dim3(nbx, g->n_groups), 256, 0, st>>>(*g, rows, mask, b1, b2, eps, bc1, bc2);
    return last_launch();
}

extern "C" gsr_status gsr_loss_l1_launch(const float *rgb, const float *depth, const float *trgb, const float *tdepth,
                                         const int32_t *tidx, int V, const gsr_raster *r, float lam, double *loss,
                                         float *grgb, float *gdepth, hipStream_t st) {
    const int64_t P = (int64_t)r->width * r->height;
    const int64_t total = (int64_t)V * P;
    const int nb = (int)(ceil_div(total, 256) < 2048 ? ceil_div(total, 256) : 2048);
    k_loss_l1<<<nb, 256, 0, st>>>(rgb, depth, trgb, tdepth, tidx, P, V, lam, grgb, gdepth, loss);
    return last_launch();
}
