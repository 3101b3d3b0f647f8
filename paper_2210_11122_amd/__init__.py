"""MI355X-native leading-order matrix elements (gfx950 HIP kernels behind a C ABI).

``Process`` wraps a handle of libme.so; see include/me.h for the ABI."""
from .binding import Process, MeError, PROCESSES, load  # noqa: F401
