// The navigation graph over hubs and query-aware entry selection (high-tier
// graph section).
//
// Hub embeddings are unit vectors, so |a - b|^2 = 2 - 2 cos(a, b): ordering
// hubs by squared L2 distance between embeddings is ordering them by cosine.
// That lets the navigation graph and its search reuse the exact engines of
// the base index:
//   navigation graph  row i = the s hubs nearest hub i (self excluded) by
//                     (squared L2, index) = the s most cosine-similar hubs;
//                     exact kNN over the embeddings (FP64 engine);
//   hub entry         the medoid of the embeddings, which is the hub of
//                     largest cosine with the mean direction
//                     (argmin |h - mu|^2 = argmax <h, mu> for unit h);
//   entry selection   query tower -> best-first search over the hub graph
//                     (k = 1, beam L_h: the register-pool search of
//                     hubsearch.hip when L_h <= 64 and the hub table is small,
//                     else the base search kernel) -> best hub,
//                     cos = 1 - d2 / 2 -> its base id, or the medoid when the
//                     cosine is below theta.
#include <new>

#include "common.h"
#include "internal.h"
#include "knn.h"

namespace ann {
namespace {

__global__ void entry_map_kernel(const int32_t *best, const float *d2, int nq,
                                 const int32_t *hub_ids, float theta, int medoid,
                                 int32_t *entry_ids, float *score, int32_t *best_hub)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const int32_t b = best[i];
    const float cosv = 1.0f - 0.5f * d2[i];
    entry_ids[i] = (b < 0 || cosv < theta) ? medoid : hub_ids[b];
    if (score) score[i] = cosv;
    if (best_hub) best_hub[i] = b;
}

__global__ void fill_kl_kernel(int32_t *k, int32_t *L, int nq, int kv, int Lv)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    k[i] = kv;
    L[i] = Lv;
}

ann_search_plan entry_plan(const ann_entry_model &m)
{
    if (m.hub_plan.pool_cap != 0) return m.hub_plan;
    ann_search_plan p{};
    ann_default_plan(m.n_hubs, m.query_tower.dout, m.s, m.L_h, &p);
    return p;
}

}  // namespace

size_t navgraph_ws(int nh, int e, int s)
{
    return knn_workspace(nh, nh, e, s) + medoid_ws(nh, e) + 512;
}

size_t entry_select_ws(int nq, const ann_tower *w)
{
    size_t b = round_up((size_t)nq * w->dout * 4, 256);       // query embeddings
    b += round_up((size_t)nq * 4, 256) * 4;                    // k, L, best, d2
    b += 256;                                                  // search counter
    b += tower_forward_ws(nq, w) + 512;
    return b;
}

}  // namespace ann

using namespace ann;

extern "C" size_t ann_navgraph_workspace_size(int32_t n_hubs, int32_t dim, int32_t s)
{
    return navgraph_ws(n_hubs, dim, s);
}

extern "C" ann_status ann_navgraph_build(const float *hub_emb, int32_t n_hubs, int32_t dim,
                                         int32_t s, int32_t *hub_graph, int32_t *hub_entry,
                                         void *workspace, size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(hub_emb && hub_graph && hub_entry && workspace, "a required pointer is NULL");
    ANN_REQUIRE(n_hubs >= 2 && dim >= 1 && dim <= 1024, "bad n_hubs or dim");
    ANN_REQUIRE(s >= 1 && s < n_hubs, "s must be in [1, n_hubs)");
    ANN_REQUIRE(ws_bytes >= navgraph_ws(n_hubs, dim, s), "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve cv{static_cast<unsigned char *>(workspace)};
    const size_t kws = knn_workspace(n_hubs, n_hubs, dim, s);
    void *kbuf = cv.take<unsigned char>(kws);
    void *mbuf = cv.take<unsigned char>(medoid_ws(n_hubs, dim));
    ann_status r = knn_run(hub_emb, n_hubs, dim, hub_emb, n_hubs, s, true, hub_graph, nullptr,
                           nullptr, kbuf, kws, st, 2);
    if (r != ANN_OK) return r;
    return ann_medoid(hub_emb, n_hubs, dim, hub_entry, mbuf, medoid_ws(n_hubs, dim), stream);
}

// the checks on a model that need neither queries nor the device
static ann_status check_model(const ann_entry_model &m)
{
    ANN_REQUIRE(m.hub_emb && m.hub_graph && m.hub_ids, "model has a NULL pointer");
    ANN_REQUIRE(m.query_tower.din >= 1 && m.query_tower.hidden >= 1 && m.query_tower.dout >= 1,
                "model has a bad query tower shape");
    ANN_REQUIRE(m.n_hubs >= 1 && m.s >= 1, "bad hub graph shape");
    ANN_SUPPORTED(m.s <= 64, "hub graph degree must be <= 64");
    ANN_REQUIRE(m.hub_entry >= 0 && m.hub_entry < m.n_hubs, "hub_entry out of range");
    ANN_REQUIRE(m.L_h >= 1 && m.L_h <= 512, "L_h must be in [1, 512]");
    ANN_REQUIRE(m.medoid >= 0, "medoid must be >= 0");
    ANN_SUPPORTED(m.query_tower.dout % 4 == 0 && m.query_tower.dout <= 1024,
                  "embedding dim must be a multiple of 4 and <= 1024");
    ANN_REQUIRE(aligned(m.hub_emb, 16), "hub_emb must be 16-byte aligned");
    return ANN_OK;
}

extern "C" ann_status ann_entry_model_create(const ann_entry_model *desc, ann_entry_model **out)
{
    ANN_REQUIRE(desc != nullptr && out != nullptr, "a required pointer is NULL");
    *out = nullptr;
    ann_status s = check_model(*desc);
    if (s != ANN_OK) return s;
    s = validate_plan(entry_plan(*desc));
    if (s != ANN_OK) return s;
    ann_entry_model *m = new (std::nothrow) ann_entry_model(*desc);
    if (!m) return fail(ANN_ENOMEM, "out of host memory for the model handle");
    *out = m;
    return ANN_OK;
}

extern "C" void ann_entry_model_destroy(ann_entry_model *model) { delete model; }

extern "C" size_t ann_entry_workspace_size(const ann_entry_model *m, int32_t nq)
{
    return m ? entry_select_ws(nq, &m->query_tower) : 0;
}

extern "C" ann_status ann_entry_select(const ann_entry_model *m, const float *queries, int32_t nq,
                                       int32_t dim, int32_t *entry_ids, float *entry_score,
                                       int32_t *best_hub, void *workspace, size_t ws_bytes,
                                       void *stream)
{
    ANN_REQUIRE(m != nullptr, "model is NULL");
    {
        ann_status ms = check_model(*m);
        if (ms != ANN_OK) return ms;
    }
    ANN_REQUIRE(m->query_tower.din == dim, "query dim %d does not match the tower (%d)", dim,
                m->query_tower.din);
    ANN_REQUIRE(nq >= 0, "nq must be >= 0");
    ANN_REQUIRE(nq == 0 || (queries && entry_ids && workspace), "a required pointer is NULL");
    ANN_REQUIRE(ws_bytes >= entry_select_ws(nq, &m->query_tower), "workspace too small");
    const ann_search_plan plan = entry_plan(*m);
    {
        ann_status ps = validate_plan(plan);
        if (ps != ANN_OK) return ps;
        ANN_REQUIRE(plan.pool_cap >= m->L_h, "hub_plan.pool_cap %d < L_h %d", plan.pool_cap,
                    m->L_h);
        ANN_SUPPORTED(search_wave_lds(plan, m->n_hubs, m->query_tower.dout) != 0 &&
                          (size_t)plan.waves_per_block *
                                  search_wave_lds(plan, m->n_hubs, m->query_tower.dout) <=
                              (size_t)device_lds_bytes(),
                      "hub_plan does not fit the hub table on a CU");
    }
    if (nq == 0) return ANN_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int e = m->query_tower.dout;
    Carve cv{static_cast<unsigned char *>(workspace)};
    float *qemb = cv.take<float>((size_t)nq * e);
    int32_t *kk = cv.take<int32_t>((size_t)nq);
    int32_t *LL = cv.take<int32_t>((size_t)nq);
    int32_t *best = cv.take<int32_t>((size_t)nq);
    float *d2 = cv.take<float>((size_t)nq);
    uint32_t *counter = cv.take<uint32_t>(64);
    void *tws = cv.p;
    ann_status s = tower_forward_run(m->query_tower, queries, nullptr, nq, qemb, tws, st);
    if (s != ANN_OK) return s;
    const int blocks = (nq + 255) / 256;
    if (hub_search_supported(m->n_hubs, e, m->s, m->L_h)) {
        // narrow beams on a small hub graph: the register-pool search
        s = hub_search_launch(m->hub_emb, m->n_hubs, e, m->hub_graph, m->s, qemb, nq, m->hub_entry,
                              m->L_h, best, d2, nullptr, nullptr, 0, st);
    } else {
        hipLaunchKernelGGL(fill_kl_kernel, dim3(blocks), dim3(256), 0, st, kk, LL, nq, 1, m->L_h);
        ANN_LAUNCHED();
        s = search_launch(m->hub_emb, m->n_hubs, e, m->hub_graph, m->s, qemb, nq, nullptr,
                          m->hub_entry, kk, LL, 1, best, d2, nullptr, nullptr, 0, plan, counter, st);
    }
    if (s != ANN_OK) return s;
    hipLaunchKernelGGL(entry_map_kernel, dim3(blocks), dim3(256), 0, st, best, d2, nq, m->hub_ids,
                       m->theta, m->medoid, entry_ids, entry_score, best_hub);
    ANN_LAUNCHED();
    return ANN_OK;
}
