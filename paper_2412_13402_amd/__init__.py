"""MI355X-native hot path of the coupled electron-phonon real-time Boltzmann
equation: collision integrals (Methods, Eq. (e-ph), Eq. (ph-ph)) and the
adaptive ERK / MIS multirate integrators (Methods, ERK and MRI methods), as
HIP kernels for gfx950 behind the C ABI of ``include/rtbte.h``.

``rtbte`` is a thin ctypes binding of ``librtbte.so``: argument marshalling
only.  There is no CPU fallback; loading fails loudly when the library is not
built.
"""
from .rtbte import (PART_ALL, PART_EPH, PART_PHE, PART_PHPH, Context, RtbteError,  # noqa: F401
                    default_options, lib_path, load)
