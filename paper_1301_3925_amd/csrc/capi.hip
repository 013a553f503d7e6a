// Library-wide C-ABI pieces: error reporting, version, grid validation and
// the device status word helpers.
#include "common.h"

namespace adlbr {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

int check_grid(const adlbr_grid *g, GridInfo *gi) {
    if (!g) {
        set_error("grid is null");
        return ADLBR_E_INVALID;
    }
    if (g->dim != 2 && g->dim != 3) {
        set_error("grid dim must be 2 or 3 (got %d)", g->dim);
        return ADLBR_E_INVALID;
    }
    if (g->boundary != ADLBR_NEUMANN && g->boundary != ADLBR_PERIODIC &&
        g->boundary != ADLBR_REFLECT) {
        set_error("unknown boundary %d", g->boundary);
        return ADLBR_E_INVALID;
    }
    long long N = 1;
    for (int c = 0; c < g->dim; ++c) {
        if (g->n[c] < 1 || g->n[c] > (1LL << 27)) {
            set_error("grid extent n[%d] = %lld out of range", c, (long long)g->n[c]);
            return ADLBR_E_RANGE;
        }
        N *= g->n[c];
        if (N >= (1LL << 28)) {
            set_error("grid has %lld+ points; at most 2^28 - 1 supported", N);
            return ADLBR_E_RANGE;
        }
    }
    gi->dim = g->dim;
    // 0 Neumann; 1 periodic and 2 reflecting share the folded-target kernels
    gi->periodic = g->boundary == ADLBR_PERIODIC ? 1 : g->boundary == ADLBR_REFLECT ? 2 : 0;
    gi->nx = (int)g->n[0];
    gi->ny = (int)g->n[1];
    gi->nz = g->dim == 3 ? (int)g->n[2] : 1;
    gi->N = N;
    return ADLBR_OK;
}

__global__ void k_status_init(int32_t *status) {
    status[0] = 0x7fffffff;
    status[1] = 0;
}

__global__ void k_status_final(int32_t *status) {
    if (status[0] == 0x7fffffff) status[0] = -1;
}

}  // namespace adlbr

extern "C" const char *adlbr_last_error(void) { return adlbr::g_last_error.c_str(); }

extern "C" int adlbr_version(void) { return 100; }
