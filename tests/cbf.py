"""Reader for the compressed container, used by tests to compare the parts
(header fields, the stored private static model, block metadata,
per-segment streams) of two containers."""
import struct


def _varint(b, pos):
    v, sh = 0, 0
    while True:
        c = b[pos]
        pos += 1
        v |= (c & 0x7F) << sh
        sh += 7
        if not c & 0x80:
            return v, pos


def parse(blob: bytes) -> dict:
    assert blob[:4] == b"PMKC"
    h = {}
    h["version"], h["path"], h["s"], h["k"] = blob[4], blob[5], blob[6], blob[7]
    h["t"], h["bs"], h["E"] = struct.unpack_from("<HHH", blob, 8)
    h["nh"], h["opt"] = blob[14], blob[15]
    h["hidden"] = list(struct.unpack_from("<4H", blob, 16))[:h["nh"]]
    h["lr"], h["beta1"], h["beta2"], h["eps"] = struct.unpack_from("<4f", blob, 24)
    h["selector"] = blob[40]
    h["smp_ppm"], = struct.unpack_from("<I", blob, 44)
    h["seed"], = struct.unpack_from("<Q", blob, 48)
    h["static_crc"], = struct.unpack_from("<I", blob, 56)
    h["n"], = struct.unpack_from("<Q", blob, 64)
    h["n_blocks"], h["n_files"] = struct.unpack_from("<II", blob, 72)
    pos = 80
    files = []
    for _ in range(h["n_files"]):
        v, pos = _varint(blob, pos)
        files.append(v)
    s, k, bs = h["s"], h["k"], h["bs"]
    private = None
    if h["selector"] & 2:
        # the stored private static model: P FP32 values after the file table,
        # in the BiGRU static model's shape (header byte 43) or the DM's
        V = 4 ** k
        if blob[43] & 15 == 1:
            Es, gh, gl = blob[60], blob[61], blob[43] >> 4
            gd, = struct.unpack_from("<H", blob, 62)
            P = V * Es + sum(2 * (3 * gh * (Es if l == 0 else 2 * gh) + 3 * gh * gh + 6 * gh) for l in range(gl))
            P += 2 * gh * gd + gd + gd * V + V
        else:
            dims = [h["t"] * h["E"]] + h["hidden"] + [V]
            P = V * h["E"] + sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1))
        private = blob[pos:pos + 4 * P]
        assert len(private) == 4 * P
        pos += 4 * P
    h["meta_start"] = pos
    blocks = []
    for _ in range(h["n_blocks"]):
        b = {}
        b["raw_len"], pos = _varint(blob, pos)
        nr, pos = _varint(blob, pos)
        runs, prev = [], 0
        for _ in range(nr):
            g, pos = _varint(blob, pos)
            ln, pos = _varint(blob, pos)
            runs.append((prev + g, ln))
            prev += g + ln
        b["runs"] = runs
        nb = b["raw_len"] - sum(x[1] for x in runs)
        l = (nb - k) // s + 1 if nb >= k else 0
        L, rem = l // bs, l % bs
        tail = nb - ((l - 1) * s + k if l else 0)
        b.update(nb=nb, l=l, L=L, rem=rem, tail=tail)
        eb = (2 * tail + 2 * k * rem + 7) // 8
        b["extras"] = blob[pos:pos + eb]
        pos += eb
        seg = []
        if L > 0:
            for _ in range(bs):
                v, pos = _varint(blob, pos)
                seg.append(v)
        b["seg_bytes"] = seg
        blocks.append(b)
    for b in blocks:
        b["streams"] = []
        for n in b["seg_bytes"]:
            b["streams"].append(blob[pos:pos + n])
            pos += n
    assert pos == len(blob), (pos, len(blob))
    return {"header": h, "files": files, "blocks": blocks, "private": private}
