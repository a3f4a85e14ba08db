"""MI355X-native hybrid FFT beamformer for CHIME/FRB (Ng et al., arXiv:1702.04728).

The hot path -- 4+4-bit decode, zero-padded N-S FFT beams clamped to the
desired pointings, E-W exact phasing, 16-point up-channelisation, Stokes I and
integration to 0.983 ms -- runs in hand-written HIP kernels for gfx950 inside
``libbeamform.so`` (C ABI in ``include/beamform.h``).  This package is the
thin Python binding over it.
"""
from .beamform import (  # noqa: F401
    BF_OK, EXPORTED, FP16_MFMA, FP32_FFT, FP32_MFMA, LIB_PATH, N_BEAMS, N_INPUTS, N_UPCHAN,
    STREAM_JOIN, STREAM_LEAVE, STREAM_MAX_SLOTS, Beamformer, BeamformError, compute_lut,
    load_library, stream_schedule,
)
