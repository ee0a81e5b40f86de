"""MI355X-native quantum quasi-Monte Carlo (arXiv:2002.12372): the order-n
charge coefficient of a wide-band Anderson dot, evaluated on gfx950.

``qqmc`` is the thin binding of the C ABI declared in ``include/qqmc.h``;
``build`` compiles the HIP library in place."""
from . import qqmc  # noqa: F401
