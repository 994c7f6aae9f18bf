// All-pairs co-occurrence (association rule mining, Section 4.3).
#include "fc_internal.h"

using namespace fc;

extern "C" int fc_pairs(fc_db *db, const int32_t *items, int32_t ni, double minsup, int32_t *gram,
                        fc_pair_rec *out, int64_t cap, int64_t *n_out, void *stream) {
    (void)db; (void)items; (void)ni; (void)minsup; (void)gram; (void)out; (void)cap;
    (void)n_out; (void)stream;
    clear_error();
    set_error("fc_pairs: not available in this build");
    return FC_ERR_INVALID;
}
