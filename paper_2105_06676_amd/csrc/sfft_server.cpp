// Batched and serving entry points -- placeholder until the batch executor lands.
#include "../../include/stencil_fft.h"
#include "sfft_runtime.h"

extern "C" {
int stencil_fft_batch(const sfft_problem*, int, void*) { return SFFT_EUNSUPPORTED; }
int sfft_server_create(sfft_server**, int, uint64_t, int) { return SFFT_EUNSUPPORTED; }
int sfft_server_submit(sfft_server*, const sfft_problem*, uint64_t*) { return SFFT_EUNSUPPORTED; }
int sfft_server_poll(sfft_server*, uint64_t, int*) { return SFFT_EUNSUPPORTED; }
int sfft_server_wait(sfft_server*, uint64_t) { return SFFT_EUNSUPPORTED; }
int sfft_server_stats(sfft_server*, char*, int64_t) { return SFFT_EUNSUPPORTED; }
void sfft_server_destroy(sfft_server*) {}
}
