// placeholder: weighted TV proximal mapping (filled in below)
#include "../../include/bq.h"
extern "C" {
struct bq_prox { int dummy; };
bq_status bq_prox_create(int, int, int, int, void*, bq_prox** out) { if (out) *out = nullptr; return BQ_EUNSUPPORTED; }
bq_status bq_prox_destroy(bq_prox*) { return BQ_OK; }
const char* bq_prox_last_error(const bq_prox*) { return "not built"; }
bq_status bq_wprox(bq_prox*, const void*, double, const void*, double, int, int, int, void*, void*, bq_prox_stats*) { return BQ_EUNSUPPORTED; }
}
