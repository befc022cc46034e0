// Entry points whose kernels live in later translation units of this library.
#include "tpc_internal.h"

extern "C" {

int tpc_track_timeframe(tpc_ctx_t* c, const tpc_clusters_t*, const tpc_geometry_t*, double, const tpc_params_t*,
                        tpc_tracks_t*, void*, int) {
    return tpc::fail(c, TPC_ERR_STATE, "time-frame path not built");
}
int tpc_timeframe_tuning(tpc_ctx_t* c, tpc_tuning_t*) { return tpc::fail(c, TPC_ERR_STATE, "not built"); }
int tpc_timeframe_set_tuning(tpc_ctx_t* c, const tpc_tuning_t*) { return tpc::fail(c, TPC_ERR_STATE, "not built"); }
}
