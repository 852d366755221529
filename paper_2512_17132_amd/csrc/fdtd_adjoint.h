// Internal interface of the discrete adjoint (fdtd_adjoint.hip).
#pragma once

#include <stdint.h>

struct fdtd_ctx;

// most steps per launch of the streaming transposed kernel (1..8, 10, 12)
constexpr int kMaxAdjTBlock = 12;

int adjoint_record_run(fdtd_ctx* c);
void adjoint_free(fdtd_ctx* c);
int64_t adjoint_bytes(const fdtd_ctx* c);
