"""Cold-start initial guess: 7x7 median filter and start parameters.

Test infrastructure only (see the package docstring).

Paper, Data Capture and Processing: the time series of normalised spectra is
treated as an image (rows = frames, columns = teeth), filtered with a 2-D
median of 7x7 footprint, and the lowest value of each filtered spectrum gives
the initial centre; the caption of the processing figure adds that the spectra
are averaged over space and time to set the other initial parameters.

Readings (the paper gives no formula for the non-centre parameters):
* edges of the image replicate the nearest row/column inside the batch;
* c0 = index of the smallest filtered value, ties to the lowest index;
* b0 = lower median over the teeth of the filtered row (order statistic
  floor((K-1)/2) counted from 0), an exact element of the row;
* d0 = clip(1 - M[c0] / b0, 0.05, 0.95), and 0.05 when b0 <= 0;
* w0 = max(2, number of teeth with M < b0 (1 - d0/2)).
The paper holds spectra in single precision, so the filtered image and the
arithmetic that decides d0 and the count behind w0 are taken in float32; every
median and minimum is an exact selection, so given the same float32 input the
whole start point is reproducible bit for bit.
"""

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def median7x7(y, chunk: int = 1024) -> np.ndarray:
    """M[f, i] = median of y[f-3..f+3, i-3..i+3] with edge replication.

    Written as the definition: pad, take every 7x7 window, take the middle
    (25th smallest) of its 49 values.
    """
    y = np.asarray(y)
    f_count, k = y.shape
    out = np.empty_like(y)
    for a in range(0, f_count, chunk):
        b = min(f_count, a + chunk)
        lo, hi = max(0, a - 3), min(f_count, b + 3)
        part = y[lo:hi]
        # rows beyond the batch edge replicate the first/last row of the batch
        top = 3 - (a - lo)
        bot = 3 - (hi - b)
        padded = np.pad(part, ((top, bot), (3, 3)), mode="edge")
        win = sliding_window_view(padded, (7, 7))        # [b-a, K, 7, 7]
        flat = win.reshape(b - a, k, 49)
        out[a:b] = np.sort(flat, axis=-1)[..., 24]
    return out


def initial_guess(y) -> np.ndarray:
    """Start point p0 = (c0, w0, d0, b0) per frame, float32 [F, 4]."""
    y32 = np.asarray(y).astype(np.float32)
    m = median7x7(y32)
    f_count, k = m.shape
    p0 = np.empty((f_count, 4), dtype=np.float32)
    r = (k - 1) // 2
    half = np.float32(0.5)
    one = np.float32(1.0)
    for f in range(f_count):
        row = m[f]
        c0 = int(np.argmin(row))                      # first minimum
        b0 = np.sort(row)[r]
        if b0 > 0:
            d0 = np.float32(one - np.float32(row[c0] / b0))
            d0 = np.float32(min(max(d0, np.float32(0.05)), np.float32(0.95)))
        else:
            d0 = np.float32(0.05)
        thr = np.float32(b0 * np.float32(one - np.float32(d0 * half)))
        w0 = max(2, int(np.count_nonzero(row < thr)))
        p0[f] = (np.float32(c0), np.float32(w0), d0, b0)
    return p0
