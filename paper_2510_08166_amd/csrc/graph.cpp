// Batched form: one frame of every view (mark -> decode -> resolve) captured
// once into a HIP graph and replayed with a single launch per frame.
#include <hip/hip_runtime.h>

#include <new>

#include "jpt.h"

struct jpt_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" jpt_status jpt_graph_capture(const jpt_scene *scene, const jpt_view *views, uint32_t n_views,
                                        uint32_t filter, jpt_frame *frame, jpt_cache *cache, uint32_t idct_mode,
                                        const jpt_tuning *tuning, void *stream, jpt_graph **out) {
    if (!out || !stream || !scene || !frame || !cache) return JPT_E_ARG;
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return JPT_E_ARG;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return JPT_E_HIP;
    jpt_status s = jpt_mark_blocks(scene, views, n_views, filter, frame, cache, tuning, stream);
    if (s == JPT_OK) s = jpt_decode_blocks(scene, frame, cache, idct_mode, tuning, stream);
    if (s == JPT_OK) s = jpt_resolve(scene, views, n_views, filter, frame, cache, tuning, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (s != JPT_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return s != JPT_OK ? s : JPT_E_HIP;
    }
    jpt_graph *h = new (std::nothrow) jpt_graph;
    if (!h) {
        (void)hipGraphDestroy(g);
        return JPT_E_HIP;
    }
    h->graph = g;
    if (hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete h;
        return JPT_E_HIP;
    }
    *out = h;
    return JPT_OK;
}

extern "C" jpt_status jpt_graph_launch(jpt_graph *g, void *stream) {
    if (!g || !g->exec) return JPT_E_ARG;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? JPT_OK : JPT_E_HIP;
}

extern "C" jpt_status jpt_graph_destroy(jpt_graph *g) {
    if (!g) return JPT_OK;
    jpt_status s = JPT_OK;
    if (g->exec && hipGraphExecDestroy(g->exec) != hipSuccess) s = JPT_E_HIP;
    if (g->graph && hipGraphDestroy(g->graph) != hipSuccess) s = JPT_E_HIP;
    delete g;
    return s;
}
