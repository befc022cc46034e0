// Entry points whose kernels live in later translation units of this library.
#include "tpc_internal.h"

extern "C" {

int tpc_track_timeframe(tpc_ctx_t* c, const tpc_clusters_t*, const tpc_geometry_t*, double, const tpc_params_t*,
                        tpc_tracks_t*, void*, int) {
    return tpc::fail(c, TPC_ERR_STATE, "time-frame path not built");
}
int tpc_timeframe_tuning(tpc_ctx_t* c, tpc_tuning_t*) { return tpc::fail(c, TPC_ERR_STATE, "not built"); }
int tpc_timeframe_set_tuning(tpc_ctx_t* c, const tpc_tuning_t*) { return tpc::fail(c, TPC_ERR_STATE, "not built"); }
int tpc_mlp_infer(tpc_ctx_t* c, const float*, int64_t, const float*, float*, void*) {
    return tpc::fail(c, TPC_ERR_STATE, "scorer not built");
}
int tpc_triplets(tpc_ctx_t* c, const tpc_clusters_t*, const tpc_geometry_t*, const tpc_params_t*, int32_t*, float*,
                 int64_t, int64_t*, void*) {
    return tpc::fail(c, TPC_ERR_STATE, "scorer not built");
}
int tpc_mlp_grad(tpc_ctx_t* c, const float*, const uint8_t*, const int32_t*, int32_t, const float*, float*, float*,
                 void*) {
    return tpc::fail(c, TPC_ERR_STATE, "scorer not built");
}
int tpc_mlp_train(tpc_ctx_t* c, const float*, const uint8_t*, const int32_t*, const tpc_train_cfg_t*, float*, float*,
                  float*, float*, void*) {
    return tpc::fail(c, TPC_ERR_STATE, "scorer not built");
}
}
