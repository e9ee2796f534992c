// Internal entry of the U-Net used by the learned solve: forward pass on a given stream.
#pragma once

#include "../../include/slnk.h"

// v [batch][2][H][W] = network(m_R, m_T) and head [batch] (may be NULL), FP32 device arrays,
// enqueued on 'stream'; EINVAL unless the network was built for height x width
slnk_status slnk_unet_forward_on(slnk_unet* u, void* stream, int batch, int height, int width, const float* m_R,
                                 const float* m_T, float* v, float* head);

// Fourier cut-off of the learned start (0: none)
int slnk_unet_start_kmax(const slnk_unet* u);
