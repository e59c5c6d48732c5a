// Serving runtime (placeholder until the continuous-batching scheduler lands).
#include "sfhad_internal.h"

extern "C" {
int sf_server_create(size_t, int, sf_server **) { return SF_ERR_UNSUPPORTED; }
int sf_mesh_register(sf_server *, const double *, int64_t, int, int, int, sf_mesh *) { return SF_ERR_UNSUPPORTED; }
int sf_submit(sf_server *, sf_mesh, int, sf_ticket *) { return SF_ERR_UNSUPPORTED; }
int sf_poll(sf_server *, sf_ticket) { return SF_ERR_UNSUPPORTED; }
int sf_wait(sf_server *, sf_ticket, const double **, double *) { return SF_ERR_UNSUPPORTED; }
int sf_release(sf_server *, sf_ticket) { return SF_ERR_UNSUPPORTED; }
int sf_mesh_unregister(sf_server *, sf_mesh) { return SF_ERR_UNSUPPORTED; }
int sf_server_destroy(sf_server *) { return SF_ERR_UNSUPPORTED; }
}
