"""MI355X-native RAK label propagation (arXiv 2301.09125): HIP kernels for
gfx950 behind the C ABI of include/lpa.h, with a thin ctypes binding."""
from .lpa import (LPA_EDEVICE, LPA_EINVAL, LPA_ENOMEM, LPA_EOVERFLOW, LPA_ETIMEDOUT,  # noqa: F401
                  LPA_ETOOLARGE, LPA_EUNSUPPORTED, LPA_NOALLOC_MAX_N, LPA_OK, LPA_ORDER_SEMISYNC, LPA_ORDER_SYNC, LPA_TIE_HASH,
                  LPA_TIE_LOWEST)
from .lpa import BatchStats, Context, LearnedStats, DeviceGraph, LpaError, Stats, default_options, library, labels_to_numpy  # noqa: F401
