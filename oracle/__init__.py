"""FP64 CPU oracle for the SwiftWRF render path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path. It shares no code
with the HIP library. See model.py for what each function follows in the paper.
"""
from . import model  # noqa: F401
from . import grad  # noqa: F401
from . import beamscan  # noqa: F401
from . import rssi  # noqa: F401
from . import ssim  # noqa: F401
from . import train  # noqa: F401
from . import paper  # noqa: F401
