// c4m_batch.hip -- batched form (many independent 2D problems per launch).
#include "c4m_internal.h"

extern "C" {
c4m_status c4m_batch_workspace_bytes(const c4m_config*, int32_t, size_t*) { return C4M_EINVAL; }
c4m_status c4m_batch_create(const c4m_config*, int32_t, void*, size_t, void*, c4m_batch**) { return C4M_EINVAL; }
c4m_status c4m_batch_problem(c4m_batch*, int32_t, c4m_problem**) { return C4M_EINVAL; }
c4m_status c4m_batch_step(c4m_batch*, int64_t) { return C4M_EINVAL; }
c4m_status c4m_batch_destroy(c4m_batch*) { return C4M_EINVAL; }
}
