"""pytest plugin (``-p tests.host.asan_plugin``) that points the CPU tests at
AddressSanitizer builds: the C ABI library named by PIC_ASAN_LIB and the
host build of the deposit arithmetic named by PIC_ASAN_DEPOSIT.  The process
must have the matching sanitizer runtime preloaded."""
import os

from paper_1606_02862_amd import _capi
from tests import host

_capi.LIB_PATH = os.environ["PIC_ASAN_LIB"]
_deposit = os.environ["PIC_ASAN_DEPOSIT"]
host.build = lambda force=False, so=None, extra=(): _deposit
