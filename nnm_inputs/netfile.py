"""Writer/reader of the binary network file used by the C library's loader.

Format (little endian):
  bytes 0..3   magic "NNMW"
  u32          version (1)
  u32          d_in  (3 or 4)
  u32          width H
  u32          n_sine K (number of sine layers; K + 1 affine layers)
  u32 x 3      reserved (0)
  float32[]    W_0, b_0, ..., W_K, b_K in the row-major [out][in] order of
               ``nnm_inputs.siren_init``.
"""

import struct

import numpy as np

from .siren_init import SirenNet, flatten_params, param_count, unflatten_params

MAGIC = b"NNMW"
VERSION = 1
HEADER = struct.Struct("<4sIIIIIII")


def write_net_file(path, net: SirenNet) -> None:
    flat = flatten_params(net.layers)
    with open(path, "wb") as fh:
        fh.write(HEADER.pack(MAGIC, VERSION, net.d_in, net.width, net.n_sine, 0, 0, 0))
        fh.write(flat.astype("<f4").tobytes())


def read_net_file(path) -> SirenNet:
    with open(path, "rb") as fh:
        raw = fh.read()
    magic, ver, d_in, width, n_sine, *_ = HEADER.unpack_from(raw, 0)
    if magic != MAGIC or ver != VERSION:
        raise ValueError("not a version-1 NNMW file")
    n = param_count(d_in, width, n_sine)
    flat = np.frombuffer(raw, dtype="<f4", count=n, offset=HEADER.size).astype(np.float32)
    return SirenNet(d_in, width, n_sine, [(W.copy(), b.copy()) for W, b in
                                          unflatten_params(flat, d_in, width, n_sine)])
