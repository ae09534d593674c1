"""MI355X-native hot path of the 1D PIC method for RICS-driven pair cascades
along magnetar field lines: a gfx950 HIP library behind a C ABI
(include/pic1d.h) and its Python binding."""
from .config import DEFAULTS, complete_config  # noqa: F401
from .pic1d import Pic1D, Pic1dError, load, lib_path, workspace_size  # noqa: F401
