// Identifiers of the lattice's lazily allocated work buffers.
#pragma once

#include "internal.hpp"

enum WorkId {
    W_APPLY_IN = 0, W_APPLY_OUT, W_APPLY_TMP,
    // FP64 solver state (two-parity fields hold even then odd)
    W_B,      // b, both parities
    W_X,      // x, both parities
    W_BHAT,   // b-hat_e
    W_R, W_RT, W_P, W_V, W_Q, W_T, W_TMP64, W_RES,   // single parity
    // inner (low precision) state
    W_IR, W_IRT, W_IP, W_IQ, W_IT, W_ITMP, W_IX,
    // gradient
    W_GLAM, W_GX, W_GN,
    W_COUNT
};
static_assert(W_COUNT <= 32, "work table too small");

int work_get(wc_lattice *lat, int id, size_t bytes, void **out);
