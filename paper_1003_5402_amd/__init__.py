"""Python binding of the MI355X column-generation DAO library (``libdao.so``).

Argument marshalling only: every step of the dose products, objective,
pricing, master and column-generation loop runs in the HIP library.  The
library must have been built (``python -m paper_1003_5402_amd.build``); there
is no fallback of any kind.  Device vectors are passed as raw device
addresses, typically ``tensor.data_ptr()`` of a torch tensor on ``cuda:0``;
the stream is a raw ``hipStream_t`` (``torch.cuda.current_stream().cuda_stream``).
"""
from __future__ import annotations

from .binding import (DAO_DFMT_AUTO, DAO_DFMT_BF16, DAO_DFMT_F16, DAO_DFMT_NATIVE, DAO_EDEVICE, DAO_EINVAL, DAO_ENOMEM,
                      DAO_EOPTIMAL, DAO_ESTALLED, DAO_ESTATE, DAO_F32, DAO_F64, DAO_MASTER_APERTURE,
                      DAO_MASTER_BEAMLET, DAO_OK, DaoError, DaoContext, Server, encode_values,
                      load_library, solve_batch, symbols, write_round_log)  # noqa: F401
