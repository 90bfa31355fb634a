"""MI355X (gfx950) probe-volume update and lossless delta packing.

Thin ctypes binding over the C ABI in ``include/probestream.h``
(``libprobestream.so``, built in-tree by :func:`build`). Every step of the
update (ray directions, trace, shade, blend, guard bands) and of the pack
(change mask, compaction, XOR byte planes, index buffer, checksum) and of
the client's unpack runs in the library's HIP kernels; this module only marshals arguments. PyTorch is
used for streams and for viewing device buffers.

If the native library is missing, importing the classes raises at first use:
there is no CPU fallback.
"""
from __future__ import annotations

from .native import (  # noqa: F401
    PV_FIRST_FRAME_NO_HISTORY, PV_KEEP_HITS, PV_MAP_FP16, PV_MAP_FP32,
    BatchGraph, Client, Context, NativeError, Receiver, Scene, Volume, build, lib, lib_path, update_probes_batched,
    volume_footprint, client_footprint, decode_yuv, yuv_dims, EXPORTED_SYMBOLS, pack_delta_noalloc,
    packet_capacity,
)
