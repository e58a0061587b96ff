#include "runtime.h"
extern "C" {
qubo_status_t qubo_server_create(size_t, int, qubo_server_t **) { qrt::set_error("server pending"); return QUBO_EINTERNAL; }
qubo_status_t qubo_server_submit(qubo_server_t *, const void *, int, qubo_dtype_t, uint64_t *) { return QUBO_EINTERNAL; }
qubo_status_t qubo_server_poll(qubo_server_t *, uint64_t, qubo_result_t *) { return QUBO_EINTERNAL; }
qubo_status_t qubo_server_wait(qubo_server_t *, uint64_t, double, qubo_result_t *) { return QUBO_EINTERNAL; }
qubo_status_t qubo_server_stats(qubo_server_t *, double *, double *, double *) { return QUBO_EINTERNAL; }
void qubo_server_destroy(qubo_server_t *) {}
}
