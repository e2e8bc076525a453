"""Minimal FITS reader for the output tests (test infrastructure): primary
HDU and IMAGE extensions with BITPIX -64/-32/8/16/32/64, written from the FITS
standard's definition of the format (2880-byte records of 80-character header
cards, big-endian data padded to a whole record)."""
import numpy as np

RECORD = 2880
_DT = {8: ">u1", 16: ">i2", 32: ">i4", 64: ">i8", -32: ">f4", -64: ">f8"}


def _value(text):
    v = text.split("/")[0].strip() if not text.strip().startswith("'") else text.strip()
    if v.startswith("'"):
        end = v.index("'", 1)
        return v[1:end].rstrip()
    if v in ("T", "F"):
        return v == "T"
    try:
        return int(v)
    except ValueError:
        return float(v)


def read(path):
    """Returns a list of (header dict, cards list, data array) per HDU."""
    raw = open(path, "rb").read()
    if len(raw) % RECORD:
        raise ValueError("file size is not a whole number of 2880-byte records")
    hdus, pos = [], 0
    while pos < len(raw):
        cards, hdr = [], {}
        while True:
            block = raw[pos:pos + RECORD]
            pos += RECORD
            done = False
            for i in range(0, RECORD, 80):
                c = block[i:i + 80].decode("ascii")
                cards.append(c)
                key = c[:8].rstrip()
                if key == "END":
                    done = True
                    break
                if c[8:10] == "= ":
                    hdr[key] = _value(c[10:])
            if done:
                break
        naxis = hdr["NAXIS"]
        shape = [hdr[f"NAXIS{k}"] for k in range(naxis, 0, -1)]
        n = int(np.prod(shape)) if naxis else 0
        dt = np.dtype(_DT[hdr["BITPIX"]])
        data = np.frombuffer(raw, dtype=dt, count=n, offset=pos).reshape(shape) if n else None
        pos += (n * dt.itemsize + RECORD - 1) // RECORD * RECORD
        hdus.append((hdr, cards, data))
    return hdus
