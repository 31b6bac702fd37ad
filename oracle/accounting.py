"""The paper's throughput and memory arithmetic.  TEST INFRASTRUCTURE.

Eq. 1: points = voxels x channels x compounding x frames (per second with a
frame rate).  Eq. 2: memory grows with voxels x frames (output) plus
channels x samples x frames (channel data); Table 4 itemises it.
"""


def points(voxels, channels, compounding, frames):
    """Eq. 1 point count: every voxel, receive channel, transmit and frame."""
    return int(voxels) * int(channels) * int(compounding) * int(frames)


def points_per_second(voxels, channels, compounding, frames, seconds):
    return points(voxels, channels, compounding, frames) / float(seconds)


def required_throughput(voxels, channels, frame_rate_hz):
    """Table 1 column: pts/s needed for a frame rate that includes compounding."""
    return int(voxels) * int(channels) * float(frame_rate_hz)


def memory_bytes(voxels, out_frames, channels, samples, in_frames, n_tx_tables=1,
                 bytes_iq=8, bytes_out=8, bytes_coord=4):
    """Table 4 itemisation (bytes): channel data, element and grid coordinates,
    arrival-time table(s), beamformed output."""
    return {
        "channel_data": channels * samples * in_frames * bytes_iq,
        "element_coords": channels * 3 * bytes_coord,
        "grid_coords": voxels * 3 * bytes_coord,
        "arrival_times": voxels * n_tx_tables * bytes_coord,
        "output": voxels * out_frames * bytes_out,
    }
