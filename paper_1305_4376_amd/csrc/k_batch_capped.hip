// k_batch_capped.hip -- the batch kernel held to 120 VGPRs, for the server's steps (see k_batch.hip).
#define TDES_BATCH_CAPPED
#include "k_batch.hip"
